// gfx950 kernels of the grid-SDF grasp step (Fast-Grasp'D, Sec. III-C and
// Sec. IV-A): forward kinematics, SDF gathers, PBD constraint corrections
// (Eq. (1)) summed per velocity test, stability/penetration/joint losses,
// the hand-written adjoint with the leaky contact gradient, and Adam.
//
// Execution model: one 64-lane wavefront owns one candidate grasp from start
// to end and walks the link-sorted contacts in 64-contact chunks. With one
// projection iteration a lane takes one (contact, test) pair, eight contacts
// per instruction, so the seven nearby gathers of a contact share cache
// lines; with several iterations a lane takes one contact and the tests run
// one after another. Every per-candidate reduction (the 7 x 6 correction
// sums, link wrenches, losses) is a wavefront reduction in a fixed order, so
// a candidate's result is bit-identical whatever else runs on the GPU. No
// workgroup barrier is used: waves never wait on each other.
#include "device_common.h"
#include "mesh_device.h"

namespace grasp {

namespace {
using namespace dev;

// per-test constants: 0..2 x, 3..11 R, 12..14 theta, 15..18 A B A' B', 19..24 Wl_bar Wa_bar

struct Ctx {
  const HandView& H;
  const SdfView& S;
  const StepConsts& P;
  float* lds;
  int lane;
  unsigned long long* groups;  // forward group counts (or null)
  const MeshView& M;           // the mesh object of a mesh step (unused on grids)
  int* face;                   // this candidate's [7][Nc] nearest faces (one-iteration mesh step, or null)
};

// Link transforms T_l (Sec. III-C, p = FK(q)): lane l composes its own
// chain (link_transform) and leaves T_l and joint l's world frame in LDS.
__device__ void forward_kinematics(const Ctx& c, const float* qb) {
  const int l = c.lane;
  if (l < c.H.L) link_transform(c.H, qb, l, c.lds + kOffT + 12 * l, c.lds + kOffJ + 6 * l);
  wave_lds_sync();
}

// Contact i of chunk ch for this lane: world position p (0 for padding).
__device__ __forceinline__ V3 contact_point(const Ctx& c, int i, int& link) {
  const HandView& H = c.H;
  const float lx = H.cx[i], ly = H.cy[i], lz = H.cz[i];
  link = H.clink[i];
  const float4* T4 = reinterpret_cast<const float4*>(c.lds + kOffT + 12 * link);
  const float4 r0 = T4[0], r1 = T4[1], r2 = T4[2];
  return xform_point(r0, r1, r2, lx, ly, lz);
}

// Per-test constants of iteration k into LDS: pose (x, theta), R(theta) and
// the rotation-derivative scalars. Poses come from the slot buffer `pose`.
__device__ void load_test_consts(const Ctx& c, const float* pose /*[7][6]*/) {
  if (c.lane < kSims) {
    const int m = c.lane;
    float* U = c.lds + kOffU + kUStride * m;
    const V3 th = v3(pose[6 * m + 3], pose[6 * m + 4], pose[6 * m + 5]);
    Rot o;
    make_rot(th, o);
    U[0] = pose[6 * m]; U[1] = pose[6 * m + 1]; U[2] = pose[6 * m + 2];
    for (int j = 0; j < 9; ++j) U[3 + j] = o.R[j];
    U[12] = th.x; U[13] = th.y; U[14] = th.z;
    U[15] = o.A; U[16] = o.B; U[17] = o.Ap; U[18] = o.Bp;
  }
  wave_lds_sync();
}

__device__ __forceinline__ void load_rot(const float* U, Rot& o) {
  for (int j = 0; j < 9; ++j) o.R[j] = U[3 + j];
  o.th = v3(U[12], U[13], U[14]);
  o.A = U[15]; o.B = U[16]; o.Ap = U[17]; o.Bp = U[18];
}

// ---------------------------------------------------------------------------
// Projection passes. Lanes take (contact, test) pairs: lane = 7 * contact +
// test for lanes 0..62 (lane 63 idle), nine contacts per group and seven
// groups per 63-contact chunk. The seven test points of a contact lie close
// together (within about a cell at the predicted pose), so one gather
// instruction touches about half as many cache lines as with one contact per
// lane, and each lane keeps the sums of its own test only. ROT selects the
// general pose: sample at R(theta)^T (p - x) with the test's (x, theta) from
// LDS; without it (one iteration) the object is at its predicted, unrotated
// pose and the test point is p minus the test's displacement.
// ---------------------------------------------------------------------------
constexpr int kGroup = 9;                 // contacts per instruction
constexpr int kGroups = 7;                // groups per chunk
constexpr int kChunk = kGroup * kGroups;  // contacts per chunk (63)

struct LaneTest {
  int m;        // test of this lane (kSims: idle)
  int sub;      // contact within the group
  V3 off;       // test displacement: test_point(p, m, dv) = p + off
};

__device__ __forceinline__ LaneTest lane_test(int lane, float dv) {
  LaneTest t;
  t.sub = lane < kChunk ? lane / kSims : kGroup - 1;
  t.m = lane < kChunk ? lane - kSims * t.sub : kSims;
  const float sx = t.m == 0 ? -dv : (t.m == 1 ? dv : 0.0f);
  const float sy = t.m == 2 ? -dv : (t.m == 3 ? dv : 0.0f);
  const float sz = t.m == 4 ? -dv : (t.m == 5 ? dv : 0.0f);
  t.off = v3(sx, sy, sz);
  return t;
}

// World points of contacts [63 ch, 63 ch + 63) into the chunk area of LDS;
// link -1 marks entries past the last contact.
__device__ __forceinline__ void stage_chunk(const Ctx& c, int ch) {
  const int i = ch * kChunk + c.lane;
  V3 p = v3(0.0f, 0.0f, 0.0f);
  int link = -1;
  if (c.lane < kChunk && i < c.H.Nc) p = contact_point(c, i, link);
  float4* P = reinterpret_cast<float4*>(c.lds + kOffP);
  P[c.lane] = make_float4(p.x, p.y, p.z, __int_as_float(link));
  wave_lds_sync();
}

// Per-test sums of N per-lane values: lanes m, m + 7, ..., m + 56 hold test m;
// added in lane order through LDS. Lane m < 7 then stores (or adds) its N
// sums at dst + stride * m.
template <int N>
__device__ __forceinline__ void test_sums(const Ctx& c, const float v[N], float* dst, int stride, bool add) {
  float* T = c.lds + kOffP;  // [N][64], N <= 6
  for (int j = 0; j < N; ++j) T[j * kWave + c.lane] = v[j];
  wave_lds_sync();
  if (c.lane < kSims)
    for (int j = 0; j < N; ++j) {
      float t = 0.0f;
      for (int k = 0; k < kGroup; ++k) t += T[j * kWave + c.lane + kSims * k];
      float* o = dst + stride * c.lane + j;
      *o = add ? *o + t : t;
    }
  wave_lds_sync();
}

// The test's object pose of this pass for ROT lanes (LDS per-test constants;
// the idle lane borrows test 6's).
__device__ __forceinline__ const float* test_consts(const Ctx& c, const LaneTest& lt) {
  return c.lds + kOffU + kUStride * (lt.m < kSims ? lt.m : kSims - 1);
}

// All seven test points p + o (|o| <= dv along one axis, dv below the cell
// size) of a contact at p: each lies in a cell within one of p's cell per
// axis, so inside p's widened block, and at most dv closer to the grid box.
__device__ __forceinline__ bool contact_clear(const SdfView& S, V3 p, float rd, float dv) {
  float e;
  const float bm = bound_at(S, p, e);
  return fmaxf(fmaf(0.999999f, e, -1.000001f * dv), 0.0f) + (bm - rd) > 1e-6f;
}

// Coulomb friction of an active sample: dp is the displacement over the step
// of the object's material point at the contact, p - r (p the hand point, r
// its object-frame coordinates, the point's rest position); in the
// one-iteration pass (the object at its predicted pose, unturned) it is the
// test's prediction -off. Adds lambda_t (t, a x t),
// lambda_t = -min(|dp_t|, mu C) / w_t, to the lane's correction sums (none
// for a slide up to the floor kSlideMin dt v0).
__device__ __forceinline__ void add_friction(const Ctx& c, V3 dp, V3 a, V3 g, float d, bool on, float inv_Im,
                                             float W[6]) {
  if (!on) return;
  Fric f;
  if (!friction_dir(g, dp, a, inv_Im, kSlideMin * (c.P.dt * c.P.v0), f)) return;
  const float mc = -c.P.mu * d;  // mu C, C = -d > 0
  const float delta = f.tl <= mc ? f.tl : mc;
  const float lam = -delta * rcp(f.wt);
  W[0] = fmaf(lam, f.th.x, W[0]);
  W[1] = fmaf(lam, f.th.y, W[1]);
  W[2] = fmaf(lam, f.th.z, W[2]);
  W[3] = fmaf(lam, f.ut.x, W[3]);
  W[4] = fmaf(lam, f.ut.y, W[4]);
  W[5] = fmaf(lam, f.ut.z, W[5]);
}

// Adjoint of add_friction for one sample: from the test's seeds (WlB, WaB),
// the contributions to d_bar, and, for a penetrating sample, to the
// adjoints of the gradient g, of a and of dp. A non-penetrating sample
// contributes through the leaky derivative of C only (its lambda_t is 0):
// d_bar += alpha mu lb_t / w_t.
__device__ __forceinline__ void friction_adjoint(const Ctx& c, V3 dp, V3 a, V3 g, float d, bool okw, bool pen,
                                                 float inv_Im, V3 WlB, V3 WaB, float& dbar, V3& gbar, V3& abar,
                                                 V3& dpbar) {
  if (!okw) return;
  Fric f;
  if (!friction_dir(g, dp, a, inv_Im, kSlideMin * (c.P.dt * c.P.v0), f)) return;
  const float lbt = fmaf(WlB.x, f.th.x, fmaf(WlB.y, f.th.y, fmaf(WlB.z, f.th.z, dot(WaB, f.ut))));
  const float iwt = rcp(f.wt);
  const float mu = c.P.mu;
  if (!pen) {
    dbar = fmaf(c.P.alpha * mu * lbt, iwt, dbar);
    return;
  }
  const float mc = -mu * d;
  const bool stat = f.tl <= mc;
  const float delta = stat ? f.tl : mc;
  const float lam = -delta * iwt;
  const float deltab = -lbt * iwt;
  const float wtb2 = 2.0f * lbt * delta * iwt * iwt;  // 2 w_t_bar
  // u_t = a x t; w_t = |t|^2 + |u_t|^2 / (I/m)
  const V3 utb = axpy(lam, WaB, (wtb2 * inv_Im) * f.ut);
  V3 thb = axpy(lam, WlB, wtb2 * f.th);
  abar = abar + cross(f.th, utb);
  thb = thb + cross(utb, a);
  // delta: |dp_t| (static) or mu C = -mu d (kinetic)
  const float tlb = stat ? deltab : 0.0f;
  if (!stat) dbar = fmaf(-mu, deltab, dbar);
  // t = dp_t / |dp_t|
  const float tt = dot(f.th, thb);
  const V3 dptb = axpy(tlb, f.th, f.itl * axpy(-tt, f.th, thb));
  // dp_t = dp - (dp . n) n, n = g / |g|
  const float snb = -dot(dptb, f.nh);
  const V3 nhb = axpy(snb, dp, (-f.sn) * dptb);
  const float nn = dot(f.nh, nhb);
  gbar = gbar + f.ing * axpy(-nn, f.nh, nhb);
  dpbar = dpbar + axpy(snb, f.nh, dptb);
}

template <bool ROT, bool TRACE, int LAY>
__device__ void forward_full(const Ctx& c, bool first, float& lpen, float* trace_s, int K, int k) {
  const HandView& H = c.H;
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, inv_Im = S.inv_Im;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  const LaneTest lt = lane_test(c.lane, c.P.dt * c.P.v0);
  const float4* P = reinterpret_cast<const float4*>(c.lds + kOffP);
  const int n_chunks = (H.Nc + kChunk - 1) / kChunk;
  // object pose of this lane's test: a = p - x, r = R^T a
  float R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  V3 x = v3(0.0f, 0.0f, 0.0f);
  if constexpr (ROT) {
    const float* U = test_consts(c, lt);
    x = v3(U[0], U[1], U[2]);
    for (int j = 0; j < 9; ++j) R[j] = U[3 + j];
  }
  auto test_pt = [&](V3 p) { return ROT ? p - x : p + lt.off; };
  auto frame_pt = [&](V3 a) { return ROT ? mul_t(R, a) : a; };
  float W[6] = {0, 0, 0, 0, 0, 0};
  float lp = 0.0f, na = 0.0f;
  for (int ch = 0; ch < n_chunks; ++ch) {
    stage_chunk(c, ch);
    float4 lo[2], hi[2];
    Located L[2];
    {
      const float4 P4 = P[lt.sub];
      L[0] = locate<LAY>(S, frame_pt(test_pt(v3(P4.x, P4.y, P4.z))));
      sdf_corners<LAY>(S, L[0].byte, lo[0], hi[0]);
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      if (g + 1 < kGroups) {
        const float4 Pn = P[kGroup * (g + 1) + lt.sub];
        L[(g + 1) & 1] = locate<LAY>(S, frame_pt(test_pt(v3(Pn.x, Pn.y, Pn.z))));
        sdf_corners<LAY>(S, L[(g + 1) & 1].byte, lo[(g + 1) & 1], hi[(g + 1) & 1]);
      }
      const float4 P4 = P[kGroup * g + lt.sub];
      const bool valid = __float_as_int(P4.w) >= 0 && lt.m < kSims;
      const V3 a = test_pt(v3(P4.x, P4.y, P4.z));
      Sample s;
      sample_sdf_from(S, L[g & 1], lo[g & 1], hi[g & 1], s);
      const V3 gn = ROT ? mul(R, s.n) : s.n;
      const float d = s.phi - rd;
      const bool act = valid && d < dact;
      lp = (first && valid && d < 0.0f && lt.m == kSims - 1) ? fmaf(0.5f * d, d, lp) : lp;
      const V3 u = cross(a, gn);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
      const bool on = act && w > wmin;
      const float lam = on ? d * rcp(w) : 0.0f;
      na += on ? 1.0f : 0.0f;
      W[0] = fmaf(lam, gn.x, W[0]);
      W[1] = fmaf(lam, gn.y, W[1]);
      W[2] = fmaf(lam, gn.z, W[2]);
      W[3] = fmaf(lam, u.x, W[3]);
      W[4] = fmaf(lam, u.y, W[4]);
      W[5] = fmaf(lam, u.z, W[5]);
      if (c.P.mu > 0.0f) {
        // the material point's displacement: the test's prediction, or p - r
        const V3 dp = ROT ? v3(P4.x, P4.y, P4.z) - mul_t(R, a) : -1.0f * lt.off;
        add_friction(c, dp, a, gn, d, on, inv_Im, W);
      }
      if constexpr (TRACE) {
        if (valid) {
          const int i = ch * kChunk + kGroup * g + lt.sub;
          float* o6 = trace_s + ((static_cast<size_t>(lt.m) * K + k) * H.Nc + H.perm[i]) * 6;
          o6[0] = d; o6[1] = gn.x; o6[2] = gn.y; o6[3] = gn.z; o6[4] = w; o6[5] = lam;
        }
      }
    }
  }
  test_sums<6>(c, W, c.lds + kOffWS, 6, false);
  test_sums<1>(c, &na, c.lds + kOffCnt, 1, false);
  lpen = wave_sum(lp);
}

// The untraced forward pass: a group of samples whose every lane is provably
// clear of the surface contributes exactly nothing (lambda = 0, no active
// constraint, no penetration energy), so its gathers are skipped. The live
// groups of a chunk are found first from the block minima; the corners of
// the next live group are requested before the current one is blended. The
// sums are bit-identical to the full pass's.
template <bool ROT, int LAY, bool FRIC>
__device__ void forward_culled(const Ctx& c, bool first, float& lpen) {
  const HandView& H = c.H;
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, inv_Im = S.inv_Im;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  const LaneTest lt = lane_test(c.lane, c.P.dt * c.P.v0);
  const float4* P = reinterpret_cast<const float4*>(c.lds + kOffP);
  const int n_chunks = (H.Nc + kChunk - 1) / kChunk;
  float R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  V3 x = v3(0.0f, 0.0f, 0.0f);
  if constexpr (ROT) {
    const float* U = test_consts(c, lt);
    x = v3(U[0], U[1], U[2]);
    for (int j = 0; j < 9; ++j) R[j] = U[3 + j];
  }
  auto frame_of = [&](float4 P4) {
    const V3 p = v3(P4.x, P4.y, P4.z);
    const V3 a = ROT ? p - x : p + lt.off;
    return ROT ? mul_t(R, a) : a;
  };
  float W[6] = {0, 0, 0, 0, 0, 0};
  float lp = 0.0f, na = 0.0f;
  uint32_t n_live = 0;
  // without rotation the seven tests of a contact share one bound
  const float dv = c.P.dt * c.P.v0;
  const bool per_contact = !ROT && fabsf(dv) <= 0.99f * S.h;
  for (int ch = 0; ch < n_chunks; ++ch) {
    stage_chunk(c, ch);
    uint32_t live = 0;
    if (per_contact) {
      // lane j bounds contact j of the chunk; group g holds contacts [9g, 9g + 9)
      const float4 Pj = P[c.lane];
      const bool needed = c.lane < kChunk && __float_as_int(Pj.w) >= 0 &&
                          !contact_clear(S, v3(Pj.x, Pj.y, Pj.z), rd, fabsf(dv));
      const uint64_t m = __builtin_amdgcn_ballot_w64(needed);
#pragma unroll
      for (int g = 0; g < kGroups; ++g)
        if ((m >> (kGroup * g)) & ((1ull << kGroup) - 1)) live |= 1u << g;
    } else {
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        const float4 P4 = P[kGroup * g + lt.sub];
        const bool valid = __float_as_int(P4.w) >= 0 && lt.m < kSims;
        const bool needed = valid && !provably_clear(S, frame_of(P4), rd);
        if (__builtin_amdgcn_ballot_w64(needed) != 0) live |= 1u << g;
      }
    }
    live = __builtin_amdgcn_readfirstlane(live);
    n_live += __builtin_popcount(live);
    if (live == 0) continue;
    int g = __builtin_ctz(live);
    float4 lo, hi, lo_n, hi_n;
    Located L = locate<LAY>(S, frame_of(P[kGroup * g + lt.sub])), L_n;
    sdf_corners<LAY>(S, L.byte, lo, hi);
    for (;;) {
      live &= live - 1;
      const int gn = live ? __builtin_ctz(live) : -1;
      if (gn >= 0) {
        L_n = locate<LAY>(S, frame_of(P[kGroup * gn + lt.sub]));
        sdf_corners<LAY>(S, L_n.byte, lo_n, hi_n);
      }
      const float4 P4 = P[kGroup * g + lt.sub];
      const bool valid = __float_as_int(P4.w) >= 0 && lt.m < kSims;
      const V3 p = v3(P4.x, P4.y, P4.z);
      const V3 a = ROT ? p - x : p + lt.off;
      Sample s;
      sample_sdf_from(S, L, lo, hi, s);
      const V3 gn_ = ROT ? mul(R, s.n) : s.n;
      const float d = s.phi - rd;
      const bool act = valid && d < dact;
      lp = (first && valid && d < 0.0f && lt.m == kSims - 1) ? fmaf(0.5f * d, d, lp) : lp;
      const V3 u = cross(a, gn_);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn_, gn_));
      const bool on = act && w > wmin;
      const float lam = on ? d * rcp(w) : 0.0f;
      na += on ? 1.0f : 0.0f;
      W[0] = fmaf(lam, gn_.x, W[0]);
      W[1] = fmaf(lam, gn_.y, W[1]);
      W[2] = fmaf(lam, gn_.z, W[2]);
      W[3] = fmaf(lam, u.x, W[3]);
      W[4] = fmaf(lam, u.y, W[4]);
      W[5] = fmaf(lam, u.z, W[5]);
      if (FRIC && c.P.mu > 0.0f) add_friction(c, ROT ? p - mul_t(R, a) : -1.0f * lt.off, a, gn_, d, on, inv_Im, W);
      if (gn < 0) break;
      g = gn;
      L = L_n;
      lo = lo_n;
      hi = hi_n;
    }
  }
  if (c.groups && c.lane == 0) {
    atomicAdd(c.groups, static_cast<unsigned long long>(n_live));
    atomicAdd(c.groups + 1, static_cast<unsigned long long>((H.Nc + kGroup - 1) / kGroup));
  }
  test_sums<6>(c, W, c.lds + kOffWS, 6, false);
  test_sums<1>(c, &na, c.lds + kOffCnt, 1, false);
  lpen = wave_sum(lp);
}

// One forward projection iteration over all contacts: the 7 x 6 correction
// sums W_m = sum_i lambda_i (g_i, u_i) (Eq. (1) per constraint, summed) and,
// on the rest test of the first iteration, the penetration energy.
// The forward pass on a mesh object: a sample queries the Phong signed
// distance through the hierarchy unless it provably lies outside the dilated
// surface: its distance to the root box, less the Phong bulge, is a lower
// bound on rho, and a sample with rho >= r_dil is neither active nor
// penetrating at rest, so it adds exactly nothing here (margins far above
// FP32 rounding). The traced pass queries every sample. The arithmetic
// after the sample is forward_full's.
template <bool ROT, bool TRACE>
__device__ void forward_mesh(const Ctx& c, bool first, float& lpen, float* trace_s, int K, int k) {
  const HandView& H = c.H;
  const float rd = c.P.r_dil, wmin = c.P.w_min, inv_Im = c.S.inv_Im;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  const LaneTest lt = lane_test(c.lane, c.P.dt * c.P.v0);
  const float4* P = reinterpret_cast<const float4*>(c.lds + kOffP);
  const int n_chunks = (H.Nc + kChunk - 1) / kChunk;
  float R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  V3 x = v3(0.0f, 0.0f, 0.0f);
  if constexpr (ROT) {
    const float* U = test_consts(c, lt);
    x = v3(U[0], U[1], U[2]);
    for (int j = 0; j < 9; ++j) R[j] = U[3 + j];
  }
  float W[6] = {0, 0, 0, 0, 0, 0};
  float lp = 0.0f, na = 0.0f;
  for (int ch = 0; ch < n_chunks; ++ch) {
    stage_chunk(c, ch);
    for (int g = 0; g < kGroups; ++g) {
      const float4 P4 = P[kGroup * g + lt.sub];
      const bool valid = __float_as_int(P4.w) >= 0 && lt.m < kSims;
      const V3 a = ROT ? v3(P4.x, P4.y, P4.z) - x : v3(P4.x, P4.y, P4.z) + lt.off;
      const V3 r = ROT ? mul_t(R, a) : a;
      bool query = true;
      if constexpr (!TRACE) {
        const float db = sqrtf(meshdev::box_d2(c.M.nodes[0], c.M.nodes[1], r));
        query = c.face || !(fmaf(0.999999f, db, -c.M.bulge) - rd > 1e-6f);
      }
      // the wave walks the hierarchy for all its lanes when one of them needs
      // it, so that a lane's face does not depend on which others are culled
      // (the adjoint's walk, without the face buffer, takes every lane)
      int f = -1;
      if (__builtin_amdgcn_ballot_w64(query) != 0) {
        float best;
        f = meshdev::nearest_triangle_wave(c.M, r, best, true);
      }
      meshdev::MeshSample s;
      if (query) {
        if constexpr (!TRACE && !ROT) {
          // the adjoint takes the same face instead of walking again
          if (c.face && valid) c.face[lt.m * H.Nc + ch * kChunk + kGroup * g + lt.sub] = f;
        }
        meshdev::mesh_sample_face(c.M, f, r, s);
      } else {
        s.rho = 1e30f;  // inactive, not penetrating: lambda = 0 with a zero normal
        s.n = v3(0.0f, 0.0f, 0.0f);
      }
      const V3 gn = ROT ? mul(R, s.n) : s.n;
      const float d = s.rho - rd;
      const bool act = valid && d < dact;
      lp = (first && valid && d < 0.0f && lt.m == kSims - 1) ? fmaf(0.5f * d, d, lp) : lp;
      const V3 u = cross(a, gn);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
      const bool on = act && w > wmin;
      const float lam = on ? d * rcp(w) : 0.0f;
      na += on ? 1.0f : 0.0f;
      W[0] = fmaf(lam, gn.x, W[0]);
      W[1] = fmaf(lam, gn.y, W[1]);
      W[2] = fmaf(lam, gn.z, W[2]);
      W[3] = fmaf(lam, u.x, W[3]);
      W[4] = fmaf(lam, u.y, W[4]);
      W[5] = fmaf(lam, u.z, W[5]);
      if constexpr (TRACE) {
        if (valid) {
          const int i = ch * kChunk + kGroup * g + lt.sub;
          float* o6 = trace_s + ((static_cast<size_t>(lt.m) * K + k) * H.Nc + H.perm[i]) * 6;
          o6[0] = d; o6[1] = gn.x; o6[2] = gn.y; o6[3] = gn.z; o6[4] = w; o6[5] = lam;
        }
      }
    }
  }
  test_sums<6>(c, W, c.lds + kOffWS, 6, false);
  test_sums<1>(c, &na, c.lds + kOffCnt, 1, false);
  lpen = wave_sum(lp);
}

template <bool KONE, int LAY, bool FRIC>
__device__ void forward_pass(const Ctx& c, bool first, float& lpen, float* trace_s, int K, int k) {
  lpen = 0.0f;
  if constexpr (LAY == kLayoutMesh) {
    if (trace_s) forward_mesh<!KONE, true>(c, first, lpen, trace_s, K, k);
    else forward_mesh<!KONE, false>(c, first, lpen, nullptr, K, k);
  } else {
    if (trace_s) forward_full<!KONE, true, LAY>(c, first, lpen, trace_s, K, k);
    else forward_culled<!KONE, LAY, FRIC>(c, first, lpen);
  }
  wave_lds_sync();
}

// Adds the 6 per-lane values of link l (wave sum) into the link wrench table.
__device__ __forceinline__ void flush_link(const Ctx& c, int l, const float v[6]) {
  float t[6];
  for (int j = 0; j < 6; ++j) t[j] = wave_sum(v[j]);
  if (c.lane == 0) {
    float* Wl = c.lds + kOffW + 6 * l;
    for (int j = 0; j < 6; ++j) Wl[j] += t[j];
  }
}

// One backward iteration (the adjoint of forward_lanes at iteration k), same
// lane layout. The per-test seeds (adjoints of the summed corrections) are in
// LDS. Each lane adds its sample's p_bar and p x p_bar to per-lane running
// sums of the current link, flushed (wave reductions) where the link changes;
// with pose_adj the lanes also sum the adjoint of their test's pose (-sum
// a_bar, sum theta_bar), which is added to the running pose adjoint.
template <bool ROT, int LAY, bool FRIC>
__device__ void backward_lanes(const Ctx& c, bool first, float pen_seed, bool pose_adj) {
  const HandView& H = c.H;
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, alpha = c.P.alpha, inv_Im = S.inv_Im;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  const LaneTest lt = lane_test(c.lane, c.P.dt * c.P.v0);
  const float4* P = reinterpret_cast<const float4*>(c.lds + kOffP);
  const int n_chunks = (H.Nc + kChunk - 1) / kChunk;
  // link of the last contact (contacts are sorted by link)
  const int last_link = H.clink[H.Nc - 1];
  const float* U = test_consts(c, lt);
  // seeds of this lane's test
  const V3 WlB = v3(U[19], U[20], U[21]);
  const V3 WaB = v3(U[22], U[23], U[24]);
  const float pseed = (first && lt.m == kSims - 1) ? pen_seed : 0.0f;
  Rot o;
  V3 x = v3(0.0f, 0.0f, 0.0f);
  if constexpr (ROT) {
    load_rot(U, o);
    x = v3(U[0], U[1], U[2]);
  }
  auto test_pt = [&](V3 p) { return ROT ? p - x : p + lt.off; };
  auto frame_pt = [&](V3 a) { return ROT ? mul_t(o.R, a) : a; };
  float acc[6] = {0, 0, 0, 0, 0, 0};
  float XB[6] = {0, 0, 0, 0, 0, 0};
  int cur = -1;
  for (int ch = 0; ch < n_chunks; ++ch) {
    stage_chunk(c, ch);
    float4 lo[2], hi[2];
    Located L[2];
    {
      const float4 P4 = P[lt.sub];
      L[0] = locate<LAY>(S, frame_pt(test_pt(v3(P4.x, P4.y, P4.z))));
      sdf_corners<LAY>(S, L[0].byte, lo[0], hi[0]);
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      if (g + 1 < kGroups) {
        const float4 Pn = P[kGroup * (g + 1) + lt.sub];
        L[(g + 1) & 1] = locate<LAY>(S, frame_pt(test_pt(v3(Pn.x, Pn.y, Pn.z))));
        sdf_corners<LAY>(S, L[(g + 1) & 1].byte, lo[(g + 1) & 1], hi[(g + 1) & 1]);
      }
      const float4 P4 = P[kGroup * g + lt.sub];
      const int link = __float_as_int(P4.w);
      const bool valid = link >= 0 && lt.m < kSims;
      const V3 p = v3(P4.x, P4.y, P4.z);
      const V3 a = test_pt(p);
      Sample s;
      sample_sdf_from(S, L[g & 1], lo[g & 1], hi[g & 1], s);
      const V3 gn = ROT ? mul(o.R, s.n) : s.n;
      const float d = s.phi - rd;
      const V3 u = cross(a, gn);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
      const float lb = fmaf(WlB.x, gn.x, fmaf(WlB.y, gn.y, fmaf(WlB.z, gn.z, dot(WaB, u))));
      const bool okw = valid && w > wmin;
      const bool pen = okw && d < dact;
      const float iw = rcp(w);
      // lambda = d / w where active (full derivative); dC/dd = -alpha elsewhere
      float dbar = okw ? (pen ? lb * iw : alpha * lb * iw) : 0.0f;
      dbar = (valid && d < 0.0f) ? fmaf(pseed, d, dbar) : dbar;
      V3 ab = v3(0.0f, 0.0f, 0.0f);
      V3 gbar = v3(0.0f, 0.0f, 0.0f);
      V3 dpb = v3(0.0f, 0.0f, 0.0f);
      const bool fric = FRIC && c.P.mu > 0.0f;
      if (fric)
        friction_adjoint(c, ROT ? p - mul_t(o.R, a) : -1.0f * lt.off, a, gn, d, okw, pen, inv_Im, WlB, WaB, dbar,
                         gbar, ab, dpb);
      V3 rbar = dbar * s.n;
      if (ROT && fric) rbar = rbar - dpb;  // dp = p - r: r_bar gets -dp_bar
      if (pen) {
        const float lam = d * iw;
        const float wbar2 = -2.0f * lb * lam * iw;
        const V3 ubar = axpy(lam, WaB, (wbar2 * inv_Im) * u);
        gbar = gbar + axpy(lam, WlB, wbar2 * gn);
        ab = ab + cross(gn, ubar);
        gbar = gbar + cross(ubar, a);
        rbar = rbar + hess_mul(S, s, ROT ? mul_t(o.R, gbar) : gbar);
      }
      // a_bar of the sample (exactly 0 on invalid lanes: dbar = 0, no penetration)
      const V3 pa = ab + (ROT ? mul(o.R, rbar) : rbar);
      if constexpr (ROT) {
        // the leak acts on the hand point only: a non-penetrating sample adds
        // nothing to the adjoint of the object's pose
        if (pose_adj && pen) {
          V3 thb = v3(0.0f, 0.0f, 0.0f);
          if (pen) thb = rot_vjp(o, 1.0f, s.n, gbar);
          thb = thb - rot_vjp(o, -1.0f, a, rbar);
          XB[0] -= pa.x; XB[1] -= pa.y; XB[2] -= pa.z;
          XB[3] += thb.x; XB[4] += thb.y; XB[5] += thb.z;
        }
      }
      // the hand point: through a = p - x and, with friction, through dp
      const V3 pb = (ROT && fric) ? pa + dpb : pa;
      const V3 tau = cross(p, pb);
      const float v6[6] = {pb.x, pb.y, pb.z, tau.x, tau.y, tau.z};
      // links of the group's first and last contacts (wave-uniform)
      const int lf = __builtin_amdgcn_readfirstlane(__float_as_int(P[kGroup * g].w));
      const int lz = __builtin_amdgcn_readfirstlane(__float_as_int(P[kGroup * g + kGroup - 1].w));
      if (lf < 0) continue;  // past the last contact
      const int ll = lz >= 0 ? lz : last_link;
      if (lf == ll) {
        if (lf != cur) {
          if (cur >= 0) flush_link(c, cur, acc);
          for (int j = 0; j < 6; ++j) acc[j] = 0.0f;
          cur = lf;
        }
        for (int j = 0; j < 6; ++j) acc[j] += v6[j];
      } else {
        if (cur >= 0) flush_link(c, cur, acc);
        for (int j = 0; j < 6; ++j) acc[j] = 0.0f;
        cur = -1;
        for (int l = lf; l <= ll; ++l) {
          float mv[6];
          for (int j = 0; j < 6; ++j) mv[j] = link == l ? v6[j] : 0.0f;
          flush_link(c, l, mv);
        }
      }
    }
  }
  if (cur >= 0) flush_link(c, cur, acc);
  // pose adjoint of the previous iteration: running adjoint += this pass's sums
  if (ROT && pose_adj) test_sums<6>(c, XB, c.lds + kOffU + 25, kUStride, true);
  wave_lds_sync();
}

// The backward pass on a mesh object: backward_lanes with the sample's
// Phong distance, its exact gradient (for d) and the action of the stated
// normal's derivative (for the penetrating samples' corrections) in place of
// the grid's value, gradient and Hessian. No friction.
template <bool ROT>
__device__ void backward_mesh(const Ctx& c, bool first, float pen_seed, bool pose_adj) {
  const HandView& H = c.H;
  const float rd = c.P.r_dil, wmin = c.P.w_min, alpha = c.P.alpha, inv_Im = c.S.inv_Im;
  const float dact = -kContactTol * (c.P.dt * c.P.v0);  // active below
  const LaneTest lt = lane_test(c.lane, c.P.dt * c.P.v0);
  const float4* P = reinterpret_cast<const float4*>(c.lds + kOffP);
  const int n_chunks = (H.Nc + kChunk - 1) / kChunk;
  // link of the last contact (contacts are sorted by link)
  const int last_link = H.clink[H.Nc - 1];
  const float* U = test_consts(c, lt);
  // seeds of this lane's test
  const V3 WlB = v3(U[19], U[20], U[21]);
  const V3 WaB = v3(U[22], U[23], U[24]);
  const float pseed = (first && lt.m == kSims - 1) ? pen_seed : 0.0f;
  Rot o;
  V3 x = v3(0.0f, 0.0f, 0.0f);
  if constexpr (ROT) {
    load_rot(U, o);
    x = v3(U[0], U[1], U[2]);
  }
  auto test_pt = [&](V3 p) { return ROT ? p - x : p + lt.off; };
  auto frame_pt = [&](V3 a) { return ROT ? mul_t(o.R, a) : a; };
  float acc[6] = {0, 0, 0, 0, 0, 0};
  float XB[6] = {0, 0, 0, 0, 0, 0};
  int cur = -1;
  for (int ch = 0; ch < n_chunks; ++ch) {
    stage_chunk(c, ch);
    for (int g = 0; g < kGroups; ++g) {
      const float4 P4 = P[kGroup * g + lt.sub];
      const int link = __float_as_int(P4.w);
      const bool valid = link >= 0 && lt.m < kSims;
      const V3 p = v3(P4.x, P4.y, P4.z);
      const V3 a = test_pt(p);
      meshdev::MeshSample s;
      if (!ROT && c.face) {
        // the face the forward found at this same point (any finite face on
        // lanes without a sample, whose results are multiplied by zero)
        const int f = valid ? c.face[lt.m * H.Nc + ch * kChunk + kGroup * g + lt.sub] : 0;
        meshdev::mesh_sample_face(c.M, f, frame_pt(a), s);
      } else {
        meshdev::mesh_sample_wave(c.M, frame_pt(a), s);
      }
      const V3 gn = ROT ? mul(o.R, s.n) : s.n;
      const float d = s.rho - rd;
      const V3 u = cross(a, gn);
      const float w = fmaf(dot(u, u), inv_Im, dot(gn, gn));
      const float lb = fmaf(WlB.x, gn.x, fmaf(WlB.y, gn.y, fmaf(WlB.z, gn.z, dot(WaB, u))));
      const bool okw = valid && w > wmin;
      const bool pen = okw && d < dact;
      const float iw = rcp(w);
      // lambda = d / w where active: the exact derivative of d (and the
      // penetration energy's); elsewhere the leak, dC/dd = -alpha, along the
      // stated normal as the hand point's direction
      float dbar = (okw && pen) ? lb * iw : 0.0f;
      dbar = (valid && d < 0.0f) ? fmaf(pseed, d, dbar) : dbar;
      const float leak = (okw && !pen) ? alpha * lb * iw : 0.0f;
      V3 ab = v3(0.0f, 0.0f, 0.0f);
      V3 gbar = v3(0.0f, 0.0f, 0.0f);
      V3 rbar = axpy(dbar, s.grad, leak * s.n);
      if (pen) {
        const float lam = d * iw;
        const float wbar2 = -2.0f * lb * lam * iw;
        const V3 ubar = axpy(lam, WaB, (wbar2 * inv_Im) * u);
        gbar = gbar + axpy(lam, WlB, wbar2 * gn);
        ab = ab + cross(gn, ubar);
        gbar = gbar + cross(ubar, a);
        rbar = rbar + meshdev::mesh_ngrad_t(s, c.M.alpha, ROT ? mul_t(o.R, gbar) : gbar);
      }
      // a_bar of the sample (exactly 0 on invalid lanes: dbar = 0, no penetration)
      const V3 pb = ab + (ROT ? mul(o.R, rbar) : rbar);
      if constexpr (ROT) {
        // the leak acts on the hand point only: a non-penetrating sample adds
        // nothing to the adjoint of the object's pose
        if (pose_adj && pen) {
          V3 thb = v3(0.0f, 0.0f, 0.0f);
          if (pen) thb = rot_vjp(o, 1.0f, s.n, gbar);
          thb = thb - rot_vjp(o, -1.0f, a, rbar);
          XB[0] -= pb.x; XB[1] -= pb.y; XB[2] -= pb.z;
          XB[3] += thb.x; XB[4] += thb.y; XB[5] += thb.z;
        }
      }
      const V3 tau = cross(p, pb);
      const float v6[6] = {pb.x, pb.y, pb.z, tau.x, tau.y, tau.z};
      // links of the group's first and last contacts (wave-uniform)
      const int lf = __builtin_amdgcn_readfirstlane(__float_as_int(P[kGroup * g].w));
      const int lz = __builtin_amdgcn_readfirstlane(__float_as_int(P[kGroup * g + kGroup - 1].w));
      if (lf < 0) continue;  // past the last contact
      const int ll = lz >= 0 ? lz : last_link;
      if (lf == ll) {
        if (lf != cur) {
          if (cur >= 0) flush_link(c, cur, acc);
          for (int j = 0; j < 6; ++j) acc[j] = 0.0f;
          cur = lf;
        }
        for (int j = 0; j < 6; ++j) acc[j] += v6[j];
      } else {
        if (cur >= 0) flush_link(c, cur, acc);
        for (int j = 0; j < 6; ++j) acc[j] = 0.0f;
        cur = -1;
        for (int l = lf; l <= ll; ++l) {
          float mv[6];
          for (int j = 0; j < 6; ++j) mv[j] = link == l ? v6[j] : 0.0f;
          flush_link(c, l, mv);
        }
      }
    }
  }
  if (cur >= 0) flush_link(c, cur, acc);
  // pose adjoint of the previous iteration: running adjoint += this pass's sums
  if (ROT && pose_adj) test_sums<6>(c, XB, c.lds + kOffU + 25, kUStride, true);
  wave_lds_sync();
}


template <bool KONE, int LAY, bool FRIC>
__device__ void backward_pass(const Ctx& c, bool first, float pen_seed, bool pose_adj) {
  if constexpr (LAY == kLayoutMesh) backward_mesh<!KONE>(c, first, pen_seed, pose_adj);
  else backward_lanes<!KONE, LAY, FRIC>(c, first, pen_seed, pose_adj);
}

__device__ __forceinline__ float* pose_slot(float* lds, int s) { return lds + kOffPose + s * kSims * 6; }

// Relaxation of iteration k's corrections for test m: omega over the number
// of active constraints (at least 1), as recorded in the counts table.
__device__ __forceinline__ float avg_factor(const Ctx& c, int k, int m) {
  const float n = c.lds[counts_offset(c.P.K, c.P.ckpt) + k * kSims + m];
  return c.P.omega / fmaxf(n, 1.0f);
}

// Writes pose_new = pose_old + (a W_lin, a/(I/m) W_ang), a = omega / n_active,
// for all tests from the last forward pass's sums (in LDS), and records that
// pass's counts as iteration k's.
__device__ __forceinline__ void advance_pose(const Ctx& c, const float* pold, float* pnew, int k) {
  if (c.lane < kSims) c.lds[counts_offset(c.P.K, c.P.ckpt) + k * kSims + c.lane] = c.lds[kOffCnt + c.lane];
  wave_lds_sync();
  if (c.lane < kSims * 6) {
    const int j = c.lane % 6;
    const float a = avg_factor(c, k, c.lane / 6);
    pnew[c.lane] = fmaf(j < 3 ? a : a * c.S.inv_Im, c.lds[kOffWS + c.lane], pold[c.lane]);
  }
  wave_lds_sync();
}

__device__ __forceinline__ void init_pose(const Ctx& c, float* p0) {
  const float dv = c.P.dt * c.P.v0;
  if (c.lane < kSims) {
    const V3 d = sim_dir(c.lane);
    float* p = p0 + 6 * c.lane;
    p[0] = dv * d.x; p[1] = dv * d.y; p[2] = dv * d.z; p[3] = 0.0f; p[4] = 0.0f; p[5] = 0.0f;
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// the per-candidate step
// ---------------------------------------------------------------------------
template <bool KONE, int LAY, bool FRIC>
__device__ __forceinline__ void candidate_step_lay(const StepArgs& A, int b, int kind, bool adam, float* lds) {
  const HandView& H = A.hand;
  const StepConsts& P = A.prm;
  int* face = (KONE && LAY == kLayoutMesh && A.mesh_face)
                  ? A.mesh_face + static_cast<size_t>(b) * kSims * A.hand.Nc : nullptr;
  const Ctx c{A.hand, A.sdf, A.prm, lds, lane_id(), A.fwd_groups, A.mesh, face};
  const int nd = H.n_dof;
  const int lane = c.lane;
  const float* qb = A.q + static_cast<size_t>(b) * nd;
  const float qj = lane < nd ? qb[lane] : 0.0f;
  const int K = P.K, ck = P.ckpt;
  const int nslots = K / ck + 1;
  const bool do_fwd = (kind != STEP_BWD) || A.poses == nullptr;
  const bool do_bwd = kind != STEP_FWD;
  float* gpose = A.poses ? A.poses + static_cast<size_t>(b) * kSims * nslots * 6 : nullptr;
  float* gcnt = A.poses ? A.poses + static_cast<size_t>(A.B) * kSims * nslots * 6 + static_cast<size_t>(b) * K * kSims
                        : nullptr;
  const size_t cnt_off = counts_offset(K, ck);

  forward_kinematics(c, qb);

  if (A.trace_p)
    for (int ch = 0; ch < H.n_chunks; ++ch) {
      const int i = ch * kWave + lane;
      int link;
      const V3 p = contact_point(c, i, link);
      if (i < H.Nc) {
        float* o = A.trace_p + (static_cast<size_t>(b) * H.Nc + H.perm[i]) * 3;
        o[0] = p.x; o[1] = p.y; o[2] = p.z;
      }
    }

  float lpen = 0.0f;
  // ---- forward: K projection iterations, checkpoints every ck ----
  if (do_fwd) {
    init_pose(c, pose_slot(lds, 0));
    float* cur = pose_slot(lds, nslots);  // scratch slot for iterations between checkpoints
    // copy slot 0 to the scratch slot
    if (lane < kSims * 6) cur[lane] = pose_slot(lds, 0)[lane];
    wave_lds_sync();
    for (int k = 0; k < K; ++k) {
      if (A.trace_poses && lane < kSims * 6)
        A.trace_poses[((static_cast<size_t>(b) * kSims + lane / 6) * (K + 1) + k) * 6 + lane % 6] = cur[lane];
      if constexpr (!KONE) load_test_consts(c, cur);
      float lp;
      float* ts = A.trace_samples ? A.trace_samples + static_cast<size_t>(b) * kSims * K * H.Nc * 6 : nullptr;
      forward_pass<KONE, LAY, FRIC>(c, k == 0, lp, ts, K, k);
      if (k == 0) lpen = lp;
      advance_pose(c, cur, cur, k);
      if ((k + 1) % ck == 0) {
        float* dst = pose_slot(lds, (k + 1) / ck);
        if (lane < kSims * 6) dst[lane] = cur[lane];
        wave_lds_sync();
      }
    }
    if (A.trace_poses && lane < kSims * 6)
      A.trace_poses[((static_cast<size_t>(b) * kSims + lane / 6) * (K + 1) + K) * 6 + lane % 6] = cur[lane];
    if (gpose && kind == STEP_FWD) {
      for (int t = lane; t < nslots * kSims * 6; t += kWave) gpose[t] = lds[kOffPose + t];
      for (int t = lane; t < K * kSims; t += kWave) gcnt[t] = lds[cnt_off + t];
    }
  } else {
    for (int t = lane; t < nslots * kSims * 6; t += kWave) lds[kOffPose + t] = gpose[t];
    for (int t = lane; t < K * kSims; t += kWave) lds[cnt_off + t] = gcnt[t];
    wave_lds_sync();
  }

  // ---- losses (Sec. IV-A) ----
  const float* fin = pose_slot(lds, nslots - 1);
  float mid = 0.0f, lo = 0.0f, up = 0.0f;
  if (lane >= 6 && lane < nd) {
    lo = H.qlo[lane];
    up = H.qup[lane];
    mid = 0.5f * (up + lo);
  }
  float vn = 0.0f, wn = 0.0f;
  if (lane < kSims) {
    const float* pm = fin + 6 * lane;
    const float idt = 1.0f / P.dt;
    const V3 v = idt * v3(pm[0], pm[1], pm[2]);
    const V3 om = idt * v3(pm[3], pm[4], pm[5]);
    vn = sqrtf(dot(v, v));
    wn = sqrtf(dot(om, om));
  }
  const float dm = (lane >= 6 && lane < nd) ? qj - mid : 0.0f;
  const float lim = (lane >= 6 && lane < nd) ? fmaxf(qj - up, 0.0f) + fmaxf(lo - qj, 0.0f) : 0.0f;
  const float Lstable = wave_sum(vn + wn) * (1.0f / kSims);
  const float range2 = wave_sum(dm * dm);
  const float Lrange = sqrtf(range2);
  const float Llimit = wave_sum(lim);
  if (do_fwd && kind != STEP_BWD) {
    // a configuration with a non-finite coordinate has no defined loss; the
    // grid clamp would otherwise map it to a finite corner value
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
  for (int t = lane; t < kMaxLinks * 6; t += kWave) lds[kOffW + t] = 0.0f;
  // seeds: lane m < 7 keeps dL/dx and dL/dtheta of test m after the last
  // iteration in its LDS slot U[25..30] (the running pose adjoint)
  if (lane < kSims) {
    const float cst = sL * P.w_stable / (kSims * P.dt);
    const float* pm = fin + 6 * lane;
    const V3 x = v3(pm[0], pm[1], pm[2]), th = v3(pm[3], pm[4], pm[5]);
    const float nx = sqrtf(dot(x, x)), nt = sqrtf(dot(th, th));
    // |v| = |x|/dt; its derivative is x/|x| / dt (0 at the origin)
    const float fx = nx > 0.0f ? cst / nx : 0.0f;
    const float ft = nt > 0.0f ? cst / nt : 0.0f;
    float* U = lds + kOffU + kUStride * lane;
    U[25] = fx * x.x; U[26] = fx * x.y; U[27] = fx * x.z;
    U[28] = ft * th.x; U[29] = ft * th.y; U[30] = ft * th.z;
  }
  const float pen_seed = sL * P.w_pen;
  const int nseg = K / ck;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    // replay the segment's iterations from its checkpoint (none when ck = 1)
    float* segbuf = pose_slot(lds, nslots);  // ck slots: poses seg*ck .. seg*ck+ck-1
    if constexpr (!KONE) {
      const float* ckp = pose_slot(lds, seg);
      if (lane < kSims * 6) segbuf[lane] = ckp[lane];
      wave_lds_sync();
      for (int j = 1; j < ck; ++j) {
        load_test_consts(c, segbuf + (j - 1) * kSims * 6);
        float lp;
        forward_pass<KONE, LAY, FRIC>(c, false, lp, nullptr, K, seg * ck + j - 1);
        advance_pose(c, segbuf + (j - 1) * kSims * 6, segbuf + j * kSims * 6, seg * ck + j - 1);
      }
    }
    for (int j = ck - 1; j >= 0; --j) {
      const int k = seg * ck + j;
      if constexpr (!KONE) load_test_consts(c, segbuf + j * kSims * 6);
      // seeds of this iteration's correction sums from the running adjoint
      if (lane < kSims) {
        float* U = lds + kOffU + kUStride * lane;
        const float om = avg_factor(c, k, lane), omi = om * c.S.inv_Im;
        U[19] = om * U[25]; U[20] = om * U[26]; U[21] = om * U[27];
        U[22] = omi * U[28]; U[23] = omi * U[29]; U[24] = omi * U[30];
      }
      wave_lds_sync();
      if constexpr (KONE) backward_pass<KONE, LAY, FRIC>(c, true, pen_seed, false);
      else backward_pass<KONE, LAY, FRIC>(c, k == 0, pen_seed, k > 0);
    }
  }

  // reverse sweep over the link tree: subtree sums, then joint torques
  if (lane == 0)
    for (int l = H.L - 1; l >= 1; --l) {
      const int pa = H.parent[l];
      float* src = lds + kOffW + 6 * l;
      float* dst = lds + kOffW + 6 * pa;
      for (int j = 0; j < 6; ++j) dst[j] += src[j];
    }
  wave_lds_sync();
  float gq = 0.0f;
  if (lane < nd) {
    // joint j = lane drives link l: the wrist (j < 6) drives the palm
    const int l = lane < 6 ? 0 : lane - 5;
    const float* Wl = lds + kOffW + 6 * l;
    const float* Jl = lds + kOffJ + 6 * l;
    gq = joint_torque(lane, qb, v3(Wl[0], Wl[1], Wl[2]), v3(Wl[3], Wl[4], Wl[5]), v3(Jl[0], Jl[1], Jl[2]),
                      v3(Jl[3], Jl[4], Jl[5]));
    if (lane >= 6) {
      // joint losses
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

// The gather layout of the candidate's grid selects the code path (uniform
// over the wavefront).
template <bool KONE, bool FRIC>
__device__ __forceinline__ void candidate_step(const StepArgs& A, int b, int kind, bool adam, float* lds) {
  if (A.sdf.layout == kLayoutZPairs) candidate_step_lay<KONE, kLayoutZPairs, FRIC>(A, b, kind, adam, lds);
  else candidate_step_lay<KONE, kLayoutYZQuads, FRIC>(A, b, kind, adam, lds);
}


// Locality order: candidates bucketed by the direction of the wrist from
// the grid's centre (a 4-bit-per-axis Morton code of the unit direction),
// by a counting sort in one workgroup. Order within a bucket is whatever
// the LDS atomics produce; no result depends on it.
constexpr int kOrderAxisBits = 4;
constexpr int kOrderBins = 1 << (3 * kOrderAxisBits);
constexpr int kOrderThreads = 1024;
static_assert(kOrderBins % kOrderThreads == 0, "bins split evenly over the threads");

__device__ __forceinline__ int order_key(const float* qb, V3 c) {
  const float x = qb[0] - c.x, y = qb[1] - c.y, z = qb[2] - c.z;
  const float n2 = fmaf(x, x, fmaf(y, y, z * z));
  const float s = n2 > 0.0f ? rsq(n2) : 0.0f;
  const float half = 0.5f * static_cast<float>(1 << kOrderAxisBits), top = static_cast<float>((1 << kOrderAxisBits) - 1);
  // fmaxf maps NaN to 0, so every key is a valid bucket
  const int ix = static_cast<int>(fminf(fmaxf(fmaf(x * s, half, half), 0.0f), top));
  const int iy = static_cast<int>(fminf(fmaxf(fmaf(y * s, half, half), 0.0f), top));
  const int iz = static_cast<int>(fminf(fmaxf(fmaf(z * s, half, half), 0.0f), top));
  int key = 0;
  for (int bit = 0; bit < kOrderAxisBits; ++bit)
    key |= (((ix >> bit) & 1) << (3 * bit)) | (((iy >> bit) & 1) << (3 * bit + 1)) | (((iz >> bit) & 1) << (3 * bit + 2));
  return key;
}

__device__ __forceinline__ V3 grid_centre(const SdfView& S) {
  const float hw = 0.5f * static_cast<float>(S.n - 1) * S.h;
  return v3(S.lo[0] + hw, S.lo[1] + hw, S.lo[2] + hw);
}

// One workgroup of kOrderThreads writes out[0..B) (a permutation of 0..B-1).
__device__ void order_block(const float* q, int nd, int B, V3 centre, int* out) {
  __shared__ int cnt[kOrderBins];
  __shared__ int part[kOrderThreads];
  const int tid = static_cast<int>(threadIdx.x);
  constexpr int kPer = kOrderBins / kOrderThreads;
  for (int i = tid; i < kOrderBins; i += kOrderThreads) cnt[i] = 0;
  __syncthreads();
  for (int b = tid; b < B; b += kOrderThreads) atomicAdd(&cnt[order_key(q + static_cast<size_t>(b) * nd, centre)], 1);
  __syncthreads();
  // exclusive prefix sum over the bins: per-thread runs, then a scan of the run totals
  int run = 0;
  for (int k = 0; k < kPer; ++k) run += cnt[tid * kPer + k];
  part[tid] = run;
  __syncthreads();
  for (int off = 1; off < kOrderThreads; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int base = part[tid] - run;
  for (int k = 0; k < kPer; ++k) {
    const int c = cnt[tid * kPer + k];
    cnt[tid * kPer + k] = base;
    base += c;
  }
  __syncthreads();
  for (int b = tid; b < B; b += kOrderThreads) {
    const int pos = atomicAdd(&cnt[order_key(q + static_cast<size_t>(b) * nd, centre)], 1);
    out[pos] = b;
  }
}

// The step on a mesh object: one wave per candidate, the same per-candidate
// code with the mesh's Phong distance sampled in place of the grid. The
// hierarchy walk is latency-bound, so the one-iteration form asks for four
// waves per SIMD (114 VGPRs, no spills; five, at 96 VGPRs, are slower).
template <bool KONE>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 256), amdgpu_waves_per_eu(KONE ? 4 : 3, 8)))
k_step_mesh(StepArgs A, int kind, int adam) {
  extern __shared__ float smem[];
  const int wpb = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int item = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x) * wpb + w);
  if (item >= A.B) return;
  float* lds = smem + static_cast<size_t>(w) * wave_lds_floats(A.prm.K, A.prm.ckpt);
  candidate_step_lay<KONE, kLayoutMesh, false>(A, item, kind, adam != 0, lds);
}

__global__ void __launch_bounds__(kOrderThreads) k_order(const float* q, int nd, int B, SdfView S, int* out) {
  order_block(q, nd, B, grid_centre(S), out);
}

__global__ void __launch_bounds__(kOrderThreads) k_order_batch(const BatchHeader* hdr, const BatchJob* jobs) {
  const int j = static_cast<int>(blockIdx.x);
  if (j >= hdr->n_jobs) return;
  const StepArgs& A = jobs[j].args;
  if (!A.order) return;
  order_block(A.q, A.hand.n_dof, A.B, grid_centre(A.sdf), const_cast<int*>(A.order));
}

// OCC is the minimum number of waves per SIMD the register allocation must
// allow (1 = the compiler's choice); it is the occupancy knob of the tuner.
// FRIC compiles the friction correction in (always with one iteration; with
// several, only when mu > 0: its registers cost a wave per SIMD there).
template <bool KONE, int OCC, bool FRIC>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 256), amdgpu_waves_per_eu(OCC, 8)))
k_step(StepArgs A, int kind, int adam) {
  extern __shared__ float smem[];
  const int wpb = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int item = __builtin_amdgcn_readfirstlane(xcd_block(static_cast<int>(gridDim.x)) * wpb + w);
  if (item >= A.B) return;
  const int b = A.order ? __builtin_amdgcn_readfirstlane(A.order[item]) : item;
  float* lds = smem + static_cast<size_t>(w) * wave_lds_floats(A.prm.K, A.prm.ckpt);
  candidate_step<KONE, FRIC>(A, b, kind, adam != 0, lds);
}

// Batched step: one launch covers every job of a device table, each
// candidate's fused forward, backward and Adam computed exactly as the
// single-job launch computes it. Workgroups go to the 8 XCDs round-robin;
// XCD x takes the x-th eighth of every job (in the job's locality order), so
// every XCD carries the same share of each job's work and sees one compact
// part of each job's grid. The header and table are read from device memory,
// so a graph captured for a grid of the batch's capacity serves any job set
// up to that many candidates; waves past the table exit at once.
template <bool KONE, int OCC, bool FRIC>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 256), amdgpu_waves_per_eu(OCC, 8)))
k_batch(const BatchHeader* __restrict__ hdr, const BatchJob* __restrict__ jobs, int lds_per_wave) {
  extern __shared__ float smem[];
  const int wpb = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int x = static_cast<int>(blockIdx.x) & 7;
  // wave-uniform by construction; readfirstlane lets the compiler see it
  const int t = __builtin_amdgcn_readfirstlane((static_cast<int>(blockIdx.x) >> 3) * wpb + w);
  if (t >= hdr->total8) return;
  int lo = 0, hi = hdr->n_jobs - 1;  // last job with begin8 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].begin8 <= t) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const int local = x * jobs[lo].slice + (t - jobs[lo].begin8);
  const StepArgs A = jobs[lo].args;  // one uniform copy, like a kernel argument
  if (local >= A.B) return;
  float* lds = smem + static_cast<size_t>(w) * lds_per_wave;
  const int b = A.order ? __builtin_amdgcn_readfirstlane(A.order[local]) : local;
  candidate_step<KONE, FRIC>(A, b, STEP_FUSED, true, lds);
}

__global__ void k_adam(int n, float* q, float* m, float* v, const float* g, AdamConsts c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mm = fmaf(c.b1, m[i], (1.0f - c.b1) * gi);
  const float vv = fmaf(c.b2, v[i], (1.0f - c.b2) * gi * gi);
  m[i] = mm;
  v[i] = vv;
  q[i] -= c.lr * (mm / c.c1) / (sqrtf(vv / c.c2) + c.eps);
}

// yz-quads: Q[k][j][i] = (phi(i,j,k), phi(i,j+1,k), phi(i,j,k+1), phi(i,j+1,k+1))
// for j, k < n - 1
__global__ void k_build_yzquads(const float* __restrict__ vals, int n, float4* __restrict__ Q) {
  const long long total = static_cast<long long>(n) * (n - 1) * (n - 1);
  const long long id = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int ix = static_cast<int>(id % n);
  const int iy = static_cast<int>((id / n) % (n - 1));
  const int iz = static_cast<int>(id / (static_cast<long long>(n) * (n - 1)));
  auto V = [&](int j, int k) { return vals[(static_cast<long long>(iz + k) * n + (iy + j)) * n + ix]; };
  Q[id] = make_float4(V(0, 0), V(1, 0), V(0, 1), V(1, 1));
}

// z-pairs: P[k][j][i] = (phi(i,j,k), phi(i,j,k+1)) for k < n - 1
__global__ void k_build_zpairs(const float* __restrict__ vals, int n, float2* __restrict__ P) {
  const long long plane = static_cast<long long>(n) * n;
  const long long total = plane * (n - 1);
  const long long id = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= total) return;
  P[id] = make_float2(vals[id], vals[id + plane]);
}

// Minimum over the corners of each block of kBlockCells^3 cells (vertices
// [b B, b B + B] per axis, clipped to the grid): a lower bound of the
// trilinear value anywhere in the block.
__global__ void k_build_bmin(const float* __restrict__ vals, int n, float* __restrict__ bmin) {
  const int nb = (n - 1 + kBlockCells - 1) / kBlockCells;
  const int id = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= nb * nb * nb) return;
  const int bx = id % nb, by = (id / nb) % nb, bz = id / (nb * nb);
  // vertices of the block's cells widened by one cell on every side
  float m = INFINITY;
  for (int k = max(bz * kBlockCells - 1, 0); k <= min(bz * kBlockCells + kBlockCells + 1, n - 1); ++k)
    for (int j = max(by * kBlockCells - 1, 0); j <= min(by * kBlockCells + kBlockCells + 1, n - 1); ++j)
      for (int i = max(bx * kBlockCells - 1, 0); i <= min(bx * kBlockCells + kBlockCells + 1, n - 1); ++i)
        m = fminf(m, vals[(static_cast<long long>(k) * n + j) * n + i]);
  bmin[id] = m;
}

__global__ void k_sample_points(SdfView S, int n, const float* __restrict__ r, float* __restrict__ out4,
                                float* __restrict__ hess9) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Sample s;
  sample_sdf(S, v3(r[3 * i], r[3 * i + 1], r[3 * i + 2]), s);
  out4[4 * i] = s.phi;
  out4[4 * i + 1] = s.n.x;
  out4[4 * i + 2] = s.n.y;
  out4[4 * i + 3] = s.n.z;
  if (hess9) {
    const V3 c0 = hess_mul(S, s, v3(1, 0, 0)), c1 = hess_mul(S, s, v3(0, 1, 0)), c2 = hess_mul(S, s, v3(0, 0, 1));
    float* H = hess9 + 9 * i;
    H[0] = c0.x; H[1] = c1.x; H[2] = c2.x;
    H[3] = c0.y; H[4] = c1.y; H[5] = c2.y;
    H[6] = c0.z; H[7] = c1.z; H[8] = c2.z;
  }
}

}  // namespace

namespace {
template <bool KONE, int OCC>
void launch_variant(const StepArgs& a, int kind, bool adam, int wpb, size_t lds, hipStream_t stream) {
  const int blocks = (a.B + wpb - 1) / wpb;
  if (KONE || a.prm.mu > 0.0f)
    hipLaunchKernelGGL((k_step<KONE, OCC, true>), dim3(blocks), dim3(wpb * kWave), lds, stream, a, kind, adam ? 1 : 0);
  else
    hipLaunchKernelGGL((k_step<false, OCC, false>), dim3(blocks), dim3(wpb * kWave), lds, stream, a, kind,
                       adam ? 1 : 0);
}
template <bool KONE>
void launch_occ(const StepArgs& a, int kind, bool adam, TileCfg cfg, size_t lds, hipStream_t stream) {
  switch (cfg.occ) {
    case 2: launch_variant<KONE, 2>(a, kind, adam, cfg.wpb, lds, stream); break;
    case 3: launch_variant<KONE, 3>(a, kind, adam, cfg.wpb, lds, stream); break;
    case 4: launch_variant<KONE, 4>(a, kind, adam, cfg.wpb, lds, stream); break;
    case 5: launch_variant<KONE, 5>(a, kind, adam, cfg.wpb, lds, stream); break;
    case 6: launch_variant<KONE, 6>(a, kind, adam, cfg.wpb, lds, stream); break;
    default: launch_variant<KONE, 1>(a, kind, adam, cfg.wpb, lds, stream); break;
  }
}
}  // namespace

bool valid_tile(TileCfg c) {
  return (c.wpb == 1 || c.wpb == 2 || c.wpb == 4) && (c.occ >= 1 && c.occ <= 6);
}

hipError_t launch_step(const StepArgs& a, StepKind kind, bool adam, TileCfg cfg, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  if (!valid_tile(cfg)) cfg = TileCfg{};
  const size_t lds = wave_lds_floats(a.prm.K, a.prm.ckpt) * cfg.wpb * sizeof(float);
  if (a.prm.K == 1)
    launch_occ<true>(a, static_cast<int>(kind), adam, cfg, lds, stream);
  else
    launch_occ<false>(a, static_cast<int>(kind), adam, cfg, lds, stream);
  return hipGetLastError();
}

hipError_t launch_step_mesh(const StepArgs& a, StepKind kind, bool adam, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  constexpr int kWpb = 2;
  const size_t lds = wave_lds_floats(a.prm.K, a.prm.ckpt) * kWpb * sizeof(float);
  const int blocks = (a.B + kWpb - 1) / kWpb;
  if (a.prm.K == 1)
    hipLaunchKernelGGL(k_step_mesh<true>, dim3(blocks), dim3(kWpb * kWave), lds, stream, a, static_cast<int>(kind),
                       adam ? 1 : 0);
  else
    hipLaunchKernelGGL(k_step_mesh<false>, dim3(blocks), dim3(kWpb * kWave), lds, stream, a, static_cast<int>(kind),
                       adam ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_order(const float* q, int n_dof, int B, const SdfView& S, int* order, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_order, dim3(1), dim3(kOrderThreads), 0, stream, q, n_dof, B, S, order);
  return hipGetLastError();
}

hipError_t launch_order_batch(const BatchHeader* hdr, const BatchJob* jobs, int max_jobs, hipStream_t stream) {
  if (max_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_batch, dim3(max_jobs), dim3(kOrderThreads), 0, stream, hdr, jobs);
  return hipGetLastError();
}

namespace {
template <bool KONE, int OCC>
void launch_batch_variant(const BatchHeader* hdr, const BatchJob* jobs, int blocks, int wpb, int lds_floats,
                          bool fric, hipStream_t stream) {
  const size_t lds = static_cast<size_t>(lds_floats) * wpb * sizeof(float);
  if (KONE || fric)
    hipLaunchKernelGGL((k_batch<KONE, OCC, true>), dim3(blocks), dim3(wpb * kWave), lds, stream, hdr, jobs,
                       lds_floats);
  else
    hipLaunchKernelGGL((k_batch<false, OCC, false>), dim3(blocks), dim3(wpb * kWave), lds, stream, hdr, jobs,
                       lds_floats);
}
}  // namespace

hipError_t launch_batch(const BatchHeader* hdr, const BatchJob* jobs, bool kone, bool fric, TileCfg cfg, int blocks,
                        int lds_floats, hipStream_t stream) {
  if (!valid_tile(cfg)) cfg = TileCfg{};
  switch ((kone ? 10 : 0) + cfg.occ) {
    case 12: launch_batch_variant<true, 2>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 13: launch_batch_variant<true, 3>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 14: launch_batch_variant<true, 4>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 15: launch_batch_variant<true, 5>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 16: launch_batch_variant<true, 6>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 2: launch_batch_variant<false, 2>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 3: launch_batch_variant<false, 3>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 4: launch_batch_variant<false, 4>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 5: launch_batch_variant<false, 5>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    case 6: launch_batch_variant<false, 6>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream); break;
    default:
      if (kone) launch_batch_variant<true, 1>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream);
      else launch_batch_variant<false, 1>(hdr, jobs, blocks, cfg.wpb, lds_floats, fric, stream);
  }
  return hipGetLastError();
}

hipError_t launch_adam(int n, float* q, float* m, float* v, const float* g, AdamConsts c, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, stream, n, q, m, v, g, c);
  return hipGetLastError();
}

hipError_t launch_build_gather(const float* values, int n, int layout, float4* cells, hipStream_t stream) {
  if (layout == kLayoutZPairs) {
    const long long total = static_cast<long long>(n) * n * (n - 1);
    hipLaunchKernelGGL(k_build_zpairs, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, stream, values,
                       n, reinterpret_cast<float2*>(cells));
  } else {
    const long long total = static_cast<long long>(n) * (n - 1) * (n - 1);
    hipLaunchKernelGGL(k_build_yzquads, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, stream,
                       values, n, cells);
  }
  return hipGetLastError();
}

hipError_t launch_build_bmin(const float* values, int n, float* bmin, hipStream_t stream) {
  const int nb = (n - 1 + kBlockCells - 1) / kBlockCells;
  const int total = nb * nb * nb;
  hipLaunchKernelGGL(k_build_bmin, dim3((total + 255) / 256), dim3(256), 0, stream, values, n, bmin);
  return hipGetLastError();
}

hipError_t launch_sample_points(const SdfView& s, int n, const float* r, float* out4, float* hess9,
                                hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_points, dim3((n + 255) / 256), dim3(256), 0, stream, s, n, r, out4, hess9);
  return hipGetLastError();
}

}  // namespace grasp
