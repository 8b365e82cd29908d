// The plain per-job form of the grasp step (one projection iteration): one
// coalesced kernel per stage, every intermediate in HBM, launched per job and
// per step with no graph. It computes the same quantities as the fused
// kernel (same sampler and adjoint formulas) and serves as the comparison
// baseline for the fused and batched forms.
//
// Stages: link transforms -> contact points -> SDF samples (d, g) for the 7
// tests -> constraint corrections summed per (candidate, test) -> losses and
// seeds -> per-contact adjoint -> link wrench sums -> reverse tree sweep ->
// Adam.
#include "device_common.h"

namespace grasp {
namespace {
using namespace dev;

constexpr int kBlock = 256;

struct PlainArgs {
  HandView H;
  SdfView S;
  StepConsts P;
  int B;
  const float* q;     // [B][nd]
  float* T;           // [B][L][12]
  float* J;           // [B][L][6]
  float* Pw;          // [B][Nc][3] contact points (sorted order)
  float* Sm;          // [B][7][Nc][4] samples: d, g
  float* W;           // [B][7][6] summed corrections
  float* NA;          // [B][7] active-constraint counts
  float* lpen;        // [B]
  float* seeds;       // [B][7][6] adjoints of the summed corrections
  float* PB;          // [B][Nc][3] adjoint of each contact point
  float* LW;          // [B][L][6] link force and torque adjoints
  float* loss;        // [B]
  float* terms;       // [B][4]
  float* dq;          // [B][nd]
};

__global__ void pk_links(PlainArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.B * a.H.L) return;
  const int b = t / a.H.L, l = t % a.H.L;
  link_transform(a.H, a.q + static_cast<size_t>(b) * a.H.n_dof, l, a.T + static_cast<size_t>(t) * 12,
                 a.J + static_cast<size_t>(t) * 6);
}

__global__ void pk_points(PlainArgs a) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(a.B) * a.H.Nc) return;
  const int b = static_cast<int>(t / a.H.Nc), i = static_cast<int>(t % a.H.Nc);
  const float4* T4 = reinterpret_cast<const float4*>(a.T + (static_cast<size_t>(b) * a.H.L + a.H.clink[i]) * 12);
  const V3 p = xform_point(T4[0], T4[1], T4[2], a.H.cx[i], a.H.cy[i], a.H.cz[i]);
  float* o = a.Pw + static_cast<size_t>(t) * 3;
  o[0] = p.x; o[1] = p.y; o[2] = p.z;
}

__global__ void pk_sample(PlainArgs a) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long n = static_cast<long long>(a.B) * kSims * a.H.Nc;
  if (t >= n) return;
  const int i = static_cast<int>(t % a.H.Nc);
  const long long bm = t / a.H.Nc;
  const int m = static_cast<int>(bm % kSims), b = static_cast<int>(bm / kSims);
  const float* pp = a.Pw + (static_cast<size_t>(b) * a.H.Nc + i) * 3;
  const V3 r = test_point(v3(pp[0], pp[1], pp[2]), m, a.P.dt * a.P.v0);
  Sample s;
  sample_sdf(a.S, r, s);
  reinterpret_cast<float4*>(a.Sm)[t] = make_float4(s.phi - a.P.r_dil, s.n.x, s.n.y, s.n.z);
}

// Block sum of N values in a fixed order: waves, then the 4 wave totals.
template <int N>
__device__ void block_sum(float v[N], float* sh) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0)
    for (int j = 0; j < N; ++j) sh[w * N + j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < N; ++j) {
      float s = sh[j];
      for (int k = 1; k < kBlock / kWave; ++k) s += sh[k * N + j];
      v[j] = s;
    }
}

// One block per (candidate, test): W = sum_i lambda_i (g_i, a_i x g_i) over
// penetrating contacts, their count, and the penetration energy on the rest test.
__global__ void __launch_bounds__(kBlock) pk_reduce(PlainArgs a) {
  __shared__ float sh[(kBlock / kWave) * 8];
  const int bm = blockIdx.x, b = bm / kSims, m = bm % kSims;
  const float dv = a.P.dt * a.P.v0;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < a.H.Nc; i += kBlock) {
    const float4 sm = reinterpret_cast<const float4*>(a.Sm)[static_cast<size_t>(bm) * a.H.Nc + i];
    const float d = sm.x;
    if (d < 0.0f) {
      const float* pp = a.Pw + (static_cast<size_t>(b) * a.H.Nc + i) * 3;
      const V3 ap = test_point(v3(pp[0], pp[1], pp[2]), m, dv);
      const V3 g = v3(sm.y, sm.z, sm.w);
      const V3 u = cross(ap, g);
      const float w = fmaf(dot(u, u), a.S.inv_Im, dot(g, g));
      if (d < -kContactTol * dv && w > a.P.w_min) {
        const float lam = d * rcp(w);
        acc[0] = fmaf(lam, g.x, acc[0]); acc[1] = fmaf(lam, g.y, acc[1]); acc[2] = fmaf(lam, g.z, acc[2]);
        acc[3] = fmaf(lam, u.x, acc[3]); acc[4] = fmaf(lam, u.y, acc[4]); acc[5] = fmaf(lam, u.z, acc[5]);
        acc[7] += 1.0f;
      }
      if (m == kSims - 1) acc[6] = fmaf(0.5f * d, d, acc[6]);
    }
  }
  block_sum<8>(acc, sh);
  if (threadIdx.x == 0) {
    for (int j = 0; j < 6; ++j) a.W[static_cast<size_t>(bm) * 6 + j] = acc[j];
    a.NA[bm] = acc[7];
    if (m == kSims - 1) a.lpen[b] = acc[6];
  }
}

// One thread per candidate: poses after the step, the four losses, and the
// seeds (adjoints of the summed corrections) for the backward.
__global__ void pk_loss(PlainArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  const StepConsts& P = a.P;
  const float dv = P.dt * P.v0, idt = 1.0f / P.dt;
  const float cst = P.w_stable / (kSims * P.dt);
  float ls = 0.0f;
  for (int m = 0; m < kSims; ++m) {
    const float* Wm = a.W + (static_cast<size_t>(b) * kSims + m) * 6;
    // corrections averaged over the test's active constraints, relaxed by omega
    const float om = P.omega / fmaxf(a.NA[static_cast<size_t>(b) * kSims + m], 1.0f), omi = om * a.S.inv_Im;
    const V3 d = sim_dir(m);
    const V3 x = v3(fmaf(om, Wm[0], dv * d.x), fmaf(om, Wm[1], dv * d.y), fmaf(om, Wm[2], dv * d.z));
    const V3 th = v3(omi * Wm[3], omi * Wm[4], omi * Wm[5]);
    const float nx = sqrtf(dot(x, x)), nt = sqrtf(dot(th, th));
    ls += nx * idt + nt * idt;
    const float fx = nx > 0.0f ? cst / nx : 0.0f, ft = nt > 0.0f ? cst / nt : 0.0f;
    float* sd = a.seeds + (static_cast<size_t>(b) * kSims + m) * 6;
    sd[0] = om * fx * x.x; sd[1] = om * fx * x.y; sd[2] = om * fx * x.z;
    sd[3] = omi * ft * th.x; sd[4] = omi * ft * th.y; sd[5] = omi * ft * th.z;
  }
  ls *= 1.0f / kSims;
  const float* qb = a.q + static_cast<size_t>(b) * a.H.n_dof;
  float r2 = 0.0f, lim = 0.0f;
  for (int j = 6; j < a.H.n_dof; ++j) {
    const float lo = a.H.qlo[j], up = a.H.qup[j], dm = qb[j] - 0.5f * (up + lo);
    r2 = fmaf(dm, dm, r2);
    lim += fmaxf(qb[j] - up, 0.0f) + fmaxf(lo - qb[j], 0.0f);
  }
  bool qbad = false;
  for (int j = 0; j < a.H.n_dof; ++j) qbad = qbad || !isfinite(qb[j]);
  const float lr = sqrtf(r2), lp = a.lpen[b];
  const float L = qbad ? __builtin_nanf("") : P.w_stable * ls + P.w_pen * lp + P.w_range * lr + P.w_limit * lim;
  a.loss[b] = L;
  if (a.terms) {
    a.terms[4 * b] = ls; a.terms[4 * b + 1] = lp; a.terms[4 * b + 2] = lr; a.terms[4 * b + 3] = lim;
  }
}

// One thread per (candidate, contact): adjoint of the contact point summed
// over the 7 tests. (d, g) come from the saved samples; penetrating samples
// re-gather their cell for the second derivative.
__global__ void pk_contact_bwd(PlainArgs a) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(a.B) * a.H.Nc) return;
  const int b = static_cast<int>(t / a.H.Nc), i = static_cast<int>(t % a.H.Nc);
  const StepConsts& P = a.P;
  const float dv = P.dt * P.v0, inv_Im = a.S.inv_Im;
  const float* pp = a.Pw + static_cast<size_t>(t) * 3;
  const V3 p = v3(pp[0], pp[1], pp[2]);
  V3 pbar = v3(0.0f, 0.0f, 0.0f);
  for (int m = 0; m < kSims; ++m) {
    const float4 sm = reinterpret_cast<const float4*>(a.Sm)[(static_cast<size_t>(b) * kSims + m) * a.H.Nc + i];
    const float* sd = a.seeds + (static_cast<size_t>(b) * kSims + m) * 6;
    const V3 WlB = v3(sd[0], sd[1], sd[2]), WaB = v3(sd[3], sd[4], sd[5]);
    const V3 ap = test_point(p, m, dv);
    const float d = sm.x;
    const V3 g = v3(sm.y, sm.z, sm.w);
    const V3 u = cross(ap, g);
    const float w = fmaf(dot(u, u), inv_Im, dot(g, g));
    const float lb = fmaf(WlB.x, g.x, fmaf(WlB.y, g.y, fmaf(WlB.z, g.z, dot(WaB, u))));
    float dbar = 0.0f;
    V3 abar = v3(0.0f, 0.0f, 0.0f);
    if (w > P.w_min) {
      const float iw = rcp(w);
      if (d < -kContactTol * dv) {
        const float lam = d * iw;
        dbar = lb * iw;
        const float wbar2 = -2.0f * lb * lam * iw;
        const V3 ubar = axpy(lam, WaB, (wbar2 * inv_Im) * u);
        V3 gbar = axpy(lam, WlB, wbar2 * g);
        abar = cross(g, ubar);
        gbar = gbar + cross(ubar, ap);
        Sample s;
        sample_sdf(a.S, ap, s);
        abar = abar + hess_mul(a.S, s, gbar);
      } else {
        dbar = P.alpha * lb * iw;
      }
    }
    if (m == kSims - 1 && d < 0.0f) dbar = fmaf(P.w_pen, d, dbar);
    abar = axpy(dbar, g, abar);
    pbar = pbar + abar;
  }
  float* o = a.PB + static_cast<size_t>(t) * 3;
  o[0] = pbar.x; o[1] = pbar.y; o[2] = pbar.z;
}

// One block per (candidate, link): force and torque (about the world origin)
// of the link's contact adjoints.
__global__ void __launch_bounds__(kBlock) pk_link_sum(PlainArgs a) {
  const int* link_start = a.H.link_start;
  __shared__ float sh[(kBlock / kWave) * 7];
  const int b = blockIdx.x / a.H.L, l = blockIdx.x % a.H.L;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = link_start[l] + threadIdx.x; i < link_start[l + 1]; i += kBlock) {
    const size_t o = (static_cast<size_t>(b) * a.H.Nc + i) * 3;
    const V3 p = v3(a.Pw[o], a.Pw[o + 1], a.Pw[o + 2]);
    const V3 pb = v3(a.PB[o], a.PB[o + 1], a.PB[o + 2]);
    const V3 tau = cross(p, pb);
    acc[0] += pb.x; acc[1] += pb.y; acc[2] += pb.z; acc[3] += tau.x; acc[4] += tau.y; acc[5] += tau.z;
  }
  block_sum<7>(acc, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 6; ++j) a.LW[static_cast<size_t>(blockIdx.x) * 6 + j] = acc[j];
}

// One thread per candidate: subtree sums leaf to root, joint torques, joint-loss gradients.
__global__ void pk_tree_bwd(PlainArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  const HandView& H = a.H;
  float* W = a.LW + static_cast<size_t>(b) * H.L * 6;
  for (int l = H.L - 1; l >= 1; --l)
    for (int j = 0; j < 6; ++j) W[6 * H.parent[l] + j] += W[6 * l + j];
  const float* qb = a.q + static_cast<size_t>(b) * H.n_dof;
  const float* Jb = a.J + static_cast<size_t>(b) * H.L * 6;
  float r2 = 0.0f;
  for (int j = 6; j < H.n_dof; ++j) {
    const float dm = qb[j] - 0.5f * (H.qup[j] + H.qlo[j]);
    r2 = fmaf(dm, dm, r2);
  }
  const float lr = sqrtf(r2);
  for (int j = 0; j < H.n_dof; ++j) {
    const int l = j < 6 ? 0 : j - 5;
    const float* Wl = W + 6 * l;
    const float* Jl = Jb + 6 * l;
    float gq = joint_torque(j, qb, v3(Wl[0], Wl[1], Wl[2]), v3(Wl[3], Wl[4], Wl[5]), v3(Jl[0], Jl[1], Jl[2]),
                            v3(Jl[3], Jl[4], Jl[5]));
    if (j >= 6) {
      const float dm = qb[j] - 0.5f * (H.qup[j] + H.qlo[j]);
      const float rg = lr > 0.0f ? a.P.w_range * dm / lr : 0.0f;
      const float lg = qb[j] > H.qup[j] ? a.P.w_limit : (qb[j] < H.qlo[j] ? -a.P.w_limit : 0.0f);
      gq += rg + lg;
    }
    a.dq[static_cast<size_t>(b) * H.n_dof + j] = gq;
  }
}

unsigned grid_for(long long n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Carves the intermediates out of the workspace (each 64-byte aligned);
// with ws == nullptr it only counts floats.
size_t layout(PlainArgs& a, const HandView& H, int B, float* ws) {
  const size_t b = static_cast<size_t>(B), L = H.L, Nc = H.Nc;
  size_t off = 0;
  auto take = [&](size_t n) {
    float* p = ws ? ws + off : nullptr;
    off += (n + 15) / 16 * 16;
    return p;
  };
  a.T = take(b * L * 12);
  a.J = take(b * L * 6);
  a.Pw = take(b * Nc * 3);
  a.Sm = take(b * kSims * Nc * 4);
  a.W = take(b * kSims * 6);
  a.NA = take(b * kSims);
  a.lpen = take(b);
  a.seeds = take(b * kSims * 6);
  a.PB = take(b * Nc * 3);
  a.LW = take(b * L * 6);
  a.dq = take(b * H.n_dof);
  return off;
}

}  // namespace

size_t plain_workspace_floats(const HandView& H, int B) {
  PlainArgs a{};
  return layout(a, H, B, nullptr);
}

hipError_t launch_plain_step(const HandView& H, const SdfView& S, const StepConsts& P, int B, const float* q,
                             float* loss, float* terms, float* ws, float** dq_out, hipStream_t stream) {
  PlainArgs a{};
  a.H = H;
  a.S = S;
  a.P = P;
  a.B = B;
  a.q = q;
  layout(a, H, B, ws);
  *dq_out = a.dq;
  if (B <= 0) return hipSuccess;
  const size_t b = B, L = H.L, Nc = H.Nc;
  a.loss = loss;
  a.terms = terms;
  hipLaunchKernelGGL(pk_links, dim3(grid_for(b * L)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_points, dim3(grid_for(b * Nc)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_sample, dim3(grid_for(b * kSims * Nc)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_reduce, dim3(B * kSims), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_loss, dim3(grid_for(b)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_contact_bwd, dim3(grid_for(b * Nc)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_link_sum, dim3(B * H.L), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(pk_tree_bwd, dim3(grid_for(b)), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace grasp
