// Gauss-Seidel projection of the grasp step on gfx950 (Sec. III-C: the
// Eq. (1) updates of the contact constraints applied one after another, each
// at the pose the previous ones left), with one projection iteration, its
// hand-written adjoint with the leaky contact gradient, the losses of
// Sec. IV-A and Adam; K projection iterations are K sweeps, each continuing
// from the pose the previous one left.
//
// Execution model: one wavefront per candidate; lanes hold 64 consecutive
// contacts of the link-sorted order (the sweep order). For each chunk and
// each velocity test the wave finds the first constraint, at or after the
// sweep position, that is active at the current pose (one gather round over
// the remaining lanes, culled by the block table), applies its correction,
// and continues after it; a round that finds none ends the chunk. Every
// constraint is therefore evaluated at the pose it would see in a serial
// sweep, with as many rounds as the chunk has active constraints, plus one.
//
// Backward, chunks in reverse: the chunk's sweep is replayed from its
// recorded start pose, giving the active lanes and the pose after each.
// Every lane then samples at the pose of its own turn; the active lanes, in
// reverse, turn the running pose adjoint into their point's adjoint and add
// their correction's pose derivative to it; the other lanes take the leaky
// term with the adjoint of the pose they saw (the leak reaches the hand
// point only). Point adjoints are summed per link over the seven tests and
// swept up the link tree into joint gradients.
#include "device_common.h"
#include "gs.h"

namespace grasp {
namespace {

using namespace dev;

// per-wave LDS layout (floats)
constexpr int kGT = 0;                       // [kMaxLinks][12] link transforms
constexpr int kGJ = kGT + kMaxLinks * 12;    // [kMaxLinks][6] joint world origin, axis
constexpr int kGW = kGJ + kMaxLinks * 6;     // [kMaxLinks][6] link force, torque adjoints
constexpr int kGPose = kGW + kMaxLinks * 6;  // [7][6] pose of each test
constexpr int kGBar = kGPose + kSims * 6;    // [7][6] running pose adjoint of each test
constexpr int kGScr = kGBar + kSims * 6;     // [6] replay pose
constexpr int kGZ = kGScr + 8;               // [65][6] poses of a replayed chunk sweep
constexpr int kGZB = kGZ + (kWave + 1) * 6;  // [65][6] their adjoints
constexpr int kGAct = kGZB + (kWave + 1) * 6;  // [64] applied lanes (ints)
constexpr int kGFloats = kGAct + kWave;
// The start pose of every (iteration, chunk, test) sweep goes to a global
// table [B][K][n_chunks][7][6] (written by the forward, read by the
// backward's replays).

struct GsCtx {
  const HandView& H;
  const SdfView& S;
  const StepConsts& P;
  float* lds;
  int lane;
};

// World position of the contact at sweep position i (0 for padding).
__device__ __forceinline__ V3 contact_world(const GsCtx& c, int i, int& link) {
  link = c.H.clink[i];
  const float4* T4 = reinterpret_cast<const float4*>(c.lds + kGT + 12 * link);
  return xform_point(T4[0], T4[1], T4[2], c.H.gcx[i], c.H.gcy[i], c.H.gcz[i]);
}

// Sample at object-frame point r (gathered only where live).
template <int LAY>
__device__ __forceinline__ void sample_at(const SdfView& S, V3 r, bool live, Sample& s) {
  const Located L = locate<LAY>(S, r);
  float4 lo4, hi4;
  sdf_corners<LAY>(S, live ? L.byte : kNoCell, lo4, hi4);
  sample_sdf_from(S, L, lo4, hi4, s);
}

// One Gauss-Seidel sweep over the chunk's constraints from the pose Pm (LDS,
// updated in place). With Z, the start pose goes to Z[0], the pose after the
// n-th applied correction to Z[n], its lane to act[n - 1]. Returns the mask
// of applied lanes. At most 64 rounds: each round ends the sweep or moves
// its position past the lane it applied.
template <int LAY>
__device__ unsigned long long gs_sweep(const GsCtx& c, V3 p, bool valid, float* Pm, float* Z, int* act) {
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, inv_Im = S.inv_Im, om = c.P.omega;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  if (Z && c.lane < 6) Z[c.lane] = Pm[c.lane];
  wave_lds_sync();
  unsigned long long applied = 0ull;
  int start = 0, n = 0;
  for (int round = 0; round <= kWave; ++round) {
    const V3 x = v3(Pm[0], Pm[1], Pm[2]);
    Rot o;
    make_rot(v3(Pm[3], Pm[4], Pm[5]), o);
    const V3 a = p - x;
    const V3 r = mul_t(o.R, a);
    const bool live = valid && c.lane >= start && !provably_clear(S, r, rd);
    if (__builtin_amdgcn_ballot_w64(live) == 0) break;
    Sample s;
    sample_at<LAY>(S, r, live, s);
    const V3 gn = mul(o.R, s.n);
    const float d = s.phi - rd;
    const V3 u = cross(a, gn);
    const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
    const unsigned long long on = __builtin_amdgcn_ballot_w64(live && d < dact && w > wmin);
    if (on == 0ull) break;
    const int j = __builtin_ctzll(on);
    wave_lds_sync();  // every lane has read Pm
    if (c.lane == j) {
      const float lam = d * rcp(w);
      const float ol = om * lam, oli = ol * inv_Im;
      Pm[0] = fmaf(ol, gn.x, Pm[0]);
      Pm[1] = fmaf(ol, gn.y, Pm[1]);
      Pm[2] = fmaf(ol, gn.z, Pm[2]);
      Pm[3] = fmaf(oli, u.x, Pm[3]);
      Pm[4] = fmaf(oli, u.y, Pm[4]);
      Pm[5] = fmaf(oli, u.z, Pm[5]);
      if (Z) {
        act[n] = j;
        for (int t = 0; t < 6; ++t) Z[6 * (n + 1) + t] = Pm[t];
      }
    }
    wave_lds_sync();
    applied |= 1ull << j;
    ++n;
    start = j + 1;
  }
  return applied;
}

template <int LAY>
__device__ void gs_candidate(const StepArgs& A, int b, int kind, bool adam, float* lds, float* starts) {
  const HandView& H = A.hand;
  const SdfView& S = A.sdf;
  const StepConsts& P = A.prm;
  const GsCtx c{H, S, P, lds, lane_id()};
  const int lane = c.lane, nd = H.n_dof;
  const float* qb = A.q + static_cast<size_t>(b) * nd;
  const float qj = lane < nd ? qb[lane] : 0.0f;
  const bool do_bwd = kind != STEP_FWD;
  const float rd = P.r_dil, wmin = P.w_min, inv_Im = S.inv_Im, om = P.omega;
  const int n_chunks = H.n_chunks;
  const int nk = P.K * n_chunks;  // sweeps of every test: K iterations over the chunks
  float* start_tab = starts ? starts + static_cast<size_t>(b) * nk * kSims * 6 : nullptr;

  if (lane < H.L) link_transform(H, qb, lane, lds + kGT + 12 * lane, lds + kGJ + 6 * lane);
  const float dv = P.dt * P.v0;
  if (lane < kSims) {
    const V3 dm = sim_dir(lane);
    float* pm = lds + kGPose + 6 * lane;
    pm[0] = dv * dm.x; pm[1] = dv * dm.y; pm[2] = dv * dm.z; pm[3] = 0.0f; pm[4] = 0.0f; pm[5] = 0.0f;
  }
  wave_lds_sync();

  // ---- forward: rest-pose penetration, then the sweeps of every test, K
  // iterations each continuing from the pose the last one left ----
  float lp = 0.0f;
  for (int kc = 0; kc < nk; ++kc) {
    const int ch = kc % n_chunks;
    const int i = ch * kWave + lane;
    const bool valid = i < H.Nc;
    int link;
    const V3 p = contact_world(c, i, link);
    if (kc < n_chunks) {
      const bool live = valid && !provably_clear(S, p, rd);
      if (__builtin_amdgcn_ballot_w64(live) != 0) {
        Sample s;
        sample_at<LAY>(S, p, live, s);
        const float d = s.phi - rd;
        lp = (live && d < 0.0f) ? fmaf(0.5f * d, d, lp) : lp;
      }
    }
    for (int m = 0; m < kSims; ++m) {
      float* Pm = lds + kGPose + 6 * m;
      if (do_bwd && lane < 6) start_tab[(kc * kSims + m) * 6 + lane] = Pm[lane];
      gs_sweep<LAY>(c, p, valid, Pm, nullptr, nullptr);
    }
  }
  const float lpen = wave_sum(lp);

  // ---- losses (Sec. IV-A) ----
  float mid = 0.0f, lo = 0.0f, up = 0.0f;
  if (lane >= 6 && lane < nd) {
    lo = H.qlo[lane];
    up = H.qup[lane];
    mid = 0.5f * (up + lo);
  }
  float vn = 0.0f, wn = 0.0f;
  if (lane < kSims) {
    const float* pm = lds + kGPose + 6 * lane;
    const float idt = 1.0f / P.dt;
    const V3 v = idt * v3(pm[0], pm[1], pm[2]);
    const V3 w = idt * v3(pm[3], pm[4], pm[5]);
    vn = sqrtf(dot(v, v));
    wn = sqrtf(dot(w, w));
  }
  const float dm = (lane >= 6 && lane < nd) ? qj - mid : 0.0f;
  const float lim = (lane >= 6 && lane < nd) ? fmaxf(qj - up, 0.0f) + fmaxf(lo - qj, 0.0f) : 0.0f;
  const float Lstable = wave_sum(vn + wn) * (1.0f / kSims);
  const float Lrange = sqrtf(wave_sum(dm * dm));
  const float Llimit = wave_sum(lim);
  if (kind != STEP_BWD) {
    const bool qbad = __builtin_amdgcn_ballot_w64(lane < nd && !isfinite(qj)) != 0;
    const float L = qbad ? __builtin_nanf("")
                         : P.w_stable * Lstable + P.w_pen * lpen + P.w_range * Lrange + P.w_limit * Llimit;
    if (lane == 0) {
      if (A.loss) A.loss[b] = L;
      if (A.terms) {
        A.terms[4 * b] = Lstable; A.terms[4 * b + 1] = lpen; A.terms[4 * b + 2] = Lrange; A.terms[4 * b + 3] = Llimit;
      }
      if (A.nonfinite && !isfinite(L)) atomicOr(A.nonfinite, 1);
    }
  }
  if (!do_bwd) return;

  // ---- backward ----
  const float sL = A.dloss ? A.dloss[b] : 1.0f;
  for (int t = lane; t < kMaxLinks * 6; t += kWave) lds[kGW + t] = 0.0f;
  if (lane < kSims) {
    // d L_stable / d(final pose) of test `lane`: |v| = |x| / dt, derivative x / |x| / dt (0 at 0)
    const float cst = sL * P.w_stable / (kSims * P.dt);
    const float* pm = lds + kGPose + 6 * lane;
    const V3 x = v3(pm[0], pm[1], pm[2]), th = v3(pm[3], pm[4], pm[5]);
    const float nx = sqrtf(dot(x, x)), nt = sqrtf(dot(th, th));
    const float fx = nx > 0.0f ? cst / nx : 0.0f, ft = nt > 0.0f ? cst / nt : 0.0f;
    float* pb = lds + kGBar + 6 * lane;
    pb[0] = fx * x.x; pb[1] = fx * x.y; pb[2] = fx * x.z;
    pb[3] = ft * th.x; pb[4] = ft * th.y; pb[5] = ft * th.z;
  }
  wave_lds_sync();
  const float pen_seed = sL * P.w_pen;
  const float alpha = P.alpha;
  float* Scr = lds + kGScr;
  float* Z = lds + kGZ;
  float* ZB = lds + kGZB;
  int* act = reinterpret_cast<int*>(lds + kGAct);
  for (int kc = nk - 1; kc >= 0; --kc) {
    const int ch = kc % n_chunks;
    const int i = ch * kWave + lane;
    const bool valid = i < H.Nc;
    int link;
    const V3 p = contact_world(c, i, link);
    V3 pacc = v3(0.0f, 0.0f, 0.0f);
    for (int m = 0; m < kSims; ++m) {
      // replay the chunk's sweep of test m
      if (lane < 6) Scr[lane] = start_tab[(kc * kSims + m) * 6 + lane];
      wave_lds_sync();
      const unsigned long long applied = gs_sweep<LAY>(c, p, valid, Scr, Z, act);
      const int n = __popcll(applied);
      // every lane at the pose of its turn: after the applied lanes below it
      const int k = __popcll(applied & ((1ull << lane) - 1ull));
      const float* Zk = Z + 6 * k;
      const V3 x = v3(Zk[0], Zk[1], Zk[2]);
      Rot o;
      make_rot(v3(Zk[3], Zk[4], Zk[5]), o);
      const V3 a = p - x;
      Sample s;
      sample_at<LAY>(S, mul_t(o.R, a), valid, s);
      const V3 gn = mul(o.R, s.n);
      const float d = s.phi - rd;
      const V3 u = cross(a, gn);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
      const float iw = rcp(w);
      const bool mine = (applied >> lane) & 1ull;
      // the running adjoint, then back through the applied corrections
      if (lane < 6) ZB[6 * n + lane] = lds[kGBar + 6 * m + lane];
      wave_lds_sync();
      V3 pb = v3(0.0f, 0.0f, 0.0f);
      for (int t = n; t >= 1; --t) {
        if (lane == act[t - 1]) {
          const float* zb = ZB + 6 * t;
          const V3 WlB = om * v3(zb[0], zb[1], zb[2]);
          const V3 WaB = (om * inv_Im) * v3(zb[3], zb[4], zb[5]);
          const float lb = fmaf(WlB.x, gn.x, fmaf(WlB.y, gn.y, fmaf(WlB.z, gn.z, dot(WaB, u))));
          const float lam = d * iw;
          const float wbar2 = -2.0f * lb * lam * iw;
          const V3 ubar = axpy(lam, WaB, (wbar2 * inv_Im) * u);
          V3 gbar = axpy(lam, WlB, wbar2 * gn);
          const V3 ab = cross(gn, ubar);
          gbar = gbar + cross(ubar, a);
          V3 rbar = (lb * iw) * s.n;
          rbar = rbar + hess_mul(S, s, mul_t(o.R, gbar));
          pb = ab + mul(o.R, rbar);
          const V3 thb = rot_vjp(o, 1.0f, s.n, gbar) - rot_vjp(o, -1.0f, a, rbar);
          float* zo = ZB + 6 * (t - 1);
          zo[0] = zb[0] - pb.x; zo[1] = zb[1] - pb.y; zo[2] = zb[2] - pb.z;
          zo[3] = zb[3] + thb.x; zo[4] = zb[4] + thb.y; zo[5] = zb[5] + thb.z;
        }
        wave_lds_sync();
      }
      if (lane < 6) lds[kGBar + 6 * m + lane] = ZB[lane];
      // the leaky term of the constraints not applied, with the adjoint of
      // the pose they saw
      if (!mine && valid && w > wmin) {
        const float* zb = ZB + 6 * k;
        const V3 WlB = om * v3(zb[0], zb[1], zb[2]);
        const V3 WaB = (om * inv_Im) * v3(zb[3], zb[4], zb[5]);
        const float lb = fmaf(WlB.x, gn.x, fmaf(WlB.y, gn.y, fmaf(WlB.z, gn.z, dot(WaB, u))));
        pb = mul(o.R, (alpha * lb * iw) * s.n);
      }
      pacc = pacc + pb;
      wave_lds_sync();
    }
    // rest-pose penetration (once per chunk)
    if (kc < n_chunks) {
      Sample s;
      sample_at<LAY>(S, p, valid, s);
      const float d = s.phi - rd;
      if (valid && d < 0.0f) pacc = pacc + (pen_seed * d) * s.n;
    }
    // per-link sums of (p_bar, p x p_bar) over the chunk (links sorted)
    const V3 tau = cross(p, pacc);
    const float v6[6] = {pacc.x, pacc.y, pacc.z, tau.x, tau.y, tau.z};
    const int lf = H.clink[ch * kWave];
    const int ll = H.clink[min(ch * kWave + kWave - 1, H.Nc - 1)];
    for (int l = lf; l <= ll; ++l) {
      for (int j = 0; j < 6; ++j) {
        const float sum = wave_sum(valid && link == l ? v6[j] : 0.0f);
        if (lane == 0) lds[kGW + 6 * l + j] += sum;
      }
    }
    wave_lds_sync();
  }

  // reverse sweep over the link tree: subtree sums, then joint torques
  if (lane == 0)
    for (int l = H.L - 1; l >= 1; --l) {
      const int pa = H.parent[l];
      for (int j = 0; j < 6; ++j) lds[kGW + 6 * pa + j] += lds[kGW + 6 * l + j];
    }
  wave_lds_sync();
  float gq = 0.0f;
  if (lane < nd) {
    const int l = lane < 6 ? 0 : lane - 5;
    const float* Wl = lds + kGW + 6 * l;
    const float* Jl = lds + kGJ + 6 * l;
    gq = joint_torque(lane, qb, v3(Wl[0], Wl[1], Wl[2]), v3(Wl[3], Wl[4], Wl[5]), v3(Jl[0], Jl[1], Jl[2]),
                      v3(Jl[3], Jl[4], Jl[5]));
    if (lane >= 6) {
      const float rg = Lrange > 0.0f ? P.w_range * dm / Lrange : 0.0f;
      const float lg = qj > up ? P.w_limit : (qj < lo ? -P.w_limit : 0.0f);
      gq = fmaf(sL, rg + lg, gq);
    }
  }
  if (lane < nd) {
    const size_t o = static_cast<size_t>(b) * nd + lane;
    if (A.dq) A.dq[o] = gq;
    if (adam) {
      const AdamConsts& ad = A.adam;
      const float mm = fmaf(ad.b1, A.m[o], (1.0f - ad.b1) * gq);
      const float vv = fmaf(ad.b2, A.v[o], (1.0f - ad.b2) * gq * gq);
      A.m[o] = mm;
      A.v[o] = vv;
      A.q_out[o] = qj - ad.lr * (mm / ad.c1) / (sqrtf(vv / ad.c2) + ad.eps);
    }
  }
}

__global__ void __launch_bounds__(kGsWaves * kWave) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_gs_step(StepArgs A, int kind, int adam, float* starts) {
  __shared__ float lds_all[kGsWaves * kGFloats];
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  const int b = static_cast<int>(blockIdx.x) * kGsWaves + wave;
  if (b >= A.B) return;
  float* lds = lds_all + wave * kGFloats;
  if (A.sdf.layout == kLayoutZPairs) gs_candidate<kLayoutZPairs>(A, b, kind, adam != 0, lds, starts);
  else gs_candidate<kLayoutYZQuads>(A, b, kind, adam != 0, lds, starts);
}

}  // namespace

size_t gs_scratch_floats(int B, int n_chunks, int K) {
  return static_cast<size_t>(B) * static_cast<size_t>(K) * static_cast<size_t>(n_chunks) * kSims * 6;
}

hipError_t launch_gs_step(const StepArgs& a, StepKind kind, bool adam, float* starts, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  const dim3 grid((a.B + kGsWaves - 1) / kGsWaves), block(kGsWaves * kWave);
  hipLaunchKernelGGL(k_gs_step, grid, block, 0, stream, a, static_cast<int>(kind), adam ? 1 : 0, starts);
  return hipGetLastError();
}

}  // namespace grasp
