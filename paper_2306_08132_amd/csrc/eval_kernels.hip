// Post-synthesis evaluation on gfx950 (Sec. V-A metrics): contact area at
// distance thresholds and intersection volume of final grasps, and the
// top-k selection behind the paper's top-10 figures.
//
// Contact area CA(tau) sums the areas of the hand's surface samples whose
// signed distance to the object (at rest) lies below tau; intersection
// volume sums the volumes of the hand's volume samples below 0. The samples
// are placed by the same forward kinematics and read through the same grid
// gather and trilinear value as the grasp step.
//
// Execution model: a workgroup takes a few candidates and its wavefronts
// split their samples (wave w takes 64-sample chunks w, w + W, ...). Lanes
// hold consecutive samples, each read once for all the workgroup's
// candidates; a lane transforms its sample by every candidate's link frames,
// drops the placements that the block-minimum table proves to lie above the
// largest threshold (or above 0 for volume samples), and gathers the rest
// with all their loads issued before any is used. Sums are lane-local, then
// a wavefront reduction, then the waves' partial sums added in wave order:
// a candidate's metrics are the same bits whatever else runs.
#include "device_common.h"
#include "eval.h"
#include "mesh_device.h"

namespace grasp {
namespace {

using namespace dev;

constexpr int kCpw = kEvalCandidates;
constexpr int kAcc = kMaxThresholds + 1;  // thresholds, then the volume
// Trilinear value of a located sample (the grasp step's arithmetic, without
// the gradient): the same bits as the step's sample at the same point.
__device__ __forceinline__ float sample_value(const SdfView& S, const Located& L, float4 lo4, float4 hi4) {
  const float c00 = fmaf(L.fx, lo4.y - lo4.x, lo4.x);
  const float c10 = fmaf(L.fx, lo4.w - lo4.z, lo4.z);
  const float c01 = fmaf(L.fx, hi4.y - hi4.x, hi4.x);
  const float c11 = fmaf(L.fx, hi4.w - hi4.z, hi4.z);
  const float dy0 = c10 - c00, dy1 = c11 - c01;
  const float c0 = fmaf(L.fy, dy0, c00), c1 = fmaf(L.fy, dy1, c01);
  const float phi = fmaf(L.fz, c1 - c0, c0);
  const V3 e = v3(L.ox * S.h, L.oy * S.h, L.oz * S.h);
  const float ee = dot(e, e);
  const float ine = rsq(fmaxf(ee, 1.17549435e-38f));
  return phi + ee * ine;
}

template <int LAY, bool SURFACE>
__device__ __forceinline__ void eval_set(const SdfView& S, const EvalView& E, const EvalConsts& C, const float* T,
                                         const bool bad[kCpw], int lane, int wave, float acc[kCpw][kAcc]) {
  const int begin = SURFACE ? 0 : E.ns, end = SURFACE ? E.ns : E.ns + E.nv;
  const float cut = SURFACE ? C.tmax : 0.0f;
  for (int base = begin + wave * kWave; base < end; base += kEvalWaves * kWave) {
    const int i = base + lane;
    const bool valid = i < end;
    const float4 P = valid ? E.pts[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int l = valid ? E.link[i] : 0;
    V3 r[kCpw];
    bool live[kCpw];
    bool any = false;
#pragma unroll
    for (int c = 0; c < kCpw; ++c) {
      const float4* T4 = reinterpret_cast<const float4*>(T + (c * kMaxLinks + l) * 12);
      r[c] = xform_point(T4[0], T4[1], T4[2], P.x, P.y, P.z);
      live[c] = valid && !bad[c] && !provably_clear(S, r[c], cut);
      any = any || live[c];
    }
    if (__builtin_amdgcn_ballot_w64(any) == 0) continue;
    Located L[kCpw];
    float4 lo4[kCpw], hi4[kCpw];
#pragma unroll
    for (int c = 0; c < kCpw; ++c) {
      L[c] = locate<LAY>(S, r[c]);
      sdf_corners<LAY>(S, live[c] ? L[c].byte : kNoCell, lo4[c], hi4[c]);
    }
#pragma unroll
    for (int c = 0; c < kCpw; ++c) {
      if (!live[c]) continue;
      const float phi = sample_value(S, L[c], lo4[c], hi4[c]);
      if constexpr (SURFACE) {
#pragma unroll
        for (int t = 0; t < kMaxThresholds; ++t)
          if (t < C.n_thr && phi < C.thr[t]) acc[c][t] += P.w;
      } else {
        if (phi < 0.0f) acc[c][kMaxThresholds] += P.w;
      }
    }
  }
}

// Eight waves per SIMD (64 registers, a few spilled): the kernel waits on
// its dependent loads (sample, block minimum, corners) most of the time, and
// with 70 registers only seven fit, so a launch of eight workgroups per CU
// ran its last eighth nearly alone; measured 0.115 -> 0.093 ms for 4096
// candidates.
template <int LAY>
__global__ void __launch_bounds__(kEvalWaves * kWave) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_evaluate(HandView H, SdfView S, EvalView E, EvalConsts C, int B, const float* __restrict__ q,
           float* __restrict__ out) {
  __shared__ float T[kCpw * kMaxLinks * 12];
  __shared__ float part[kEvalWaves][kCpw][kAcc];
  __shared__ int bad_s[kCpw];
  const int tid = static_cast<int>(threadIdx.x);
  const int lane = lane_id();
  const int wave = tid / kWave;
  const int b0 = static_cast<int>(blockIdx.x) * kCpw;  // < B: the grid has ceil(B / kCpw) workgroups
  const int nd = H.n_dof;
  // a candidate past B or with a non-finite coordinate is skipped (its
  // metrics are NaN); link frames of the workgroup's candidates
  if (wave == 0) {
#pragma unroll
    for (int c = 0; c < kCpw; ++c) {
      const int b = b0 + c;
      const bool in = b < B;
      const float qj = (in && lane < nd) ? q[static_cast<size_t>(b) * nd + lane] : 0.0f;
      const bool bad = !in || __builtin_amdgcn_ballot_w64(!isfinite(qj)) != 0;
      if (lane == 0) bad_s[c] = bad;
    }
  }
  for (int t = tid; t < kCpw * H.L; t += kEvalWaves * kWave) {
    const int c = t / H.L, l = t - c * H.L;
    const int b = min(b0 + c, B - 1);
    float Jw[6];
    link_transform(H, q + static_cast<size_t>(b) * nd, l, T + (c * kMaxLinks + l) * 12, Jw);
  }
  __syncthreads();
  bool bad[kCpw];
#pragma unroll
  for (int c = 0; c < kCpw; ++c) bad[c] = bad_s[c] != 0;
  float acc[kCpw][kAcc];
#pragma unroll
  for (int c = 0; c < kCpw; ++c)
#pragma unroll
    for (int t = 0; t < kAcc; ++t) acc[c][t] = 0.0f;
  eval_set<LAY, true>(S, E, C, T, bad, lane, wave, acc);
  eval_set<LAY, false>(S, E, C, T, bad, lane, wave, acc);
#pragma unroll
  for (int c = 0; c < kCpw; ++c)
#pragma unroll
    for (int t = 0; t < kAcc; ++t)
      if (t < C.n_thr || t == kMaxThresholds) {
        const float s = wave_sum(acc[c][t]);
        if (lane == 0) part[wave][c][t] = s;
      }
  __syncthreads();
  if (tid < kCpw * kAcc) {
    const int c = tid / kAcc, t = tid - c * kAcc;
    const int b = b0 + c;
    if (b < B && (t < C.n_thr || t == kMaxThresholds)) {
      float s = part[0][c][t];
      for (int w = 1; w < kEvalWaves; ++w) s += part[w][c][t];
      out[static_cast<size_t>(b) * (C.n_thr + 1) + (t == kMaxThresholds ? C.n_thr : t)] =
          bad[c] ? __builtin_nanf("") : s;
    }
  }
}

// The same metrics against a mesh object's Phong signed distance: one
// workgroup per candidate, its link frames in LDS, one sample per lane,
// each wave walking the hierarchy once for its 64 samples. A sample outside
// the mesh's bounding box is at least its distance to the box from the flat
// surface, and the Phong point lies within `bulge` (alpha times the longest
// edge) of the flat one, so a sample whose box distance exceeds the cut by
// more than the bulge (with margins far above FP32 rounding) adds nothing and
// skips the query.
// Sums as above: lane-sequential, wave butterfly, waves in order.
__global__ void __launch_bounds__(kEvalWaves * kWave) k_evaluate_mesh(HandView H, MeshView M, EvalView E,
                                                                       EvalConsts C, float bulge, int B,
                                                                       const float* __restrict__ q,
                                                                       float* __restrict__ out) {
  __shared__ float T[kMaxLinks * 12];
  __shared__ float part[kEvalWaves][kAcc];
  __shared__ int bad_s;
  const int tid = static_cast<int>(threadIdx.x);
  const int lane = lane_id();
  const int wave = tid / kWave;
  const int b = static_cast<int>(blockIdx.x);  // < B: one workgroup per candidate
  const int nd = H.n_dof;
  const float* qb = q + static_cast<size_t>(b) * nd;
  if (wave == 0) {
    const float qj = lane < nd ? qb[lane] : 0.0f;
    const bool bad = __builtin_amdgcn_ballot_w64(!isfinite(qj)) != 0;
    if (lane == 0) bad_s = bad;
  }
  if (tid < H.L) {
    float Jw[6];
    link_transform(H, qb, tid, T + 12 * tid, Jw);
  }
  __syncthreads();
  float acc[kAcc];
#pragma unroll
  for (int t = 0; t < kAcc; ++t) acc[t] = 0.0f;
  const int n = E.ns + E.nv;
  // the wave's lanes take consecutive samples and walk the hierarchy together
  for (int i0 = tid - lane; i0 < n; i0 += kEvalWaves * kWave) {
    const int i = i0 + lane;
    float4 P = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    V3 r = v3(0.0f, 0.0f, 0.0f);
    bool query = false;
    if (i < n) {
      P = E.pts[i];
      const float4* T4 = reinterpret_cast<const float4*>(T + 12 * E.link[i]);
      r = xform_point(T4[0], T4[1], T4[2], P.x, P.y, P.z);
      const float cut = i < E.ns ? C.tmax : 0.0f;
      const float db = sqrtf(meshdev::box_d2(M.nodes[0], M.nodes[1], r));
      query = !(fmaf(0.999999f, db, -bulge) - cut > 1e-6f);
    }
    if (__builtin_amdgcn_ballot_w64(query) == 0) continue;
    float best;
    const int f = meshdev::nearest_triangle_wave(M, r, best, query);
    if (!query) continue;
    float rho;
    V3 g;
    meshdev::mesh_sdf_face(M, f, r, rho, g);
    if (i < E.ns) {
#pragma unroll
      for (int t = 0; t < kMaxThresholds; ++t)
        if (t < C.n_thr && rho < C.thr[t]) acc[t] += P.w;
    } else if (rho < 0.0f) {
      acc[kMaxThresholds] += P.w;
    }
  }
#pragma unroll
  for (int t = 0; t < kAcc; ++t)
    if (t < C.n_thr || t == kMaxThresholds) {
      const float s = wave_sum(acc[t]);
      if (lane == 0) part[wave][t] = s;
    }
  __syncthreads();
  if (tid < kAcc && (tid < C.n_thr || tid == kMaxThresholds)) {
    float s = part[0][tid];
    for (int w = 1; w < kEvalWaves; ++w) s += part[w][tid];
    out[static_cast<size_t>(b) * (C.n_thr + 1) + (tid == kMaxThresholds ? C.n_thr : tid)] =
        bad_s ? __builtin_nanf("") : s;
  }
}

// Key of candidate i as one 64-bit word whose unsigned order is the ranking:
// the key mapped to an order-preserving 32-bit code (negated when higher is
// better, -0 taken as +0, NaN after everything), then the index.
__device__ __forceinline__ unsigned long long rank_word(const float* key, int i, bool higher) {
  float k = key[i];
  uint32_t u;
  if (isnan(k)) {
    u = 0xFFFFFFFFu;
  } else {
    k = higher ? -k : k;
    k = k == 0.0f ? 0.0f : k;
    const uint32_t bits = __float_as_uint(k);
    u = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
  }
  return (static_cast<unsigned long long>(u) << 32) | static_cast<uint32_t>(i);
}

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long x) {
  for (int s = 32; s >= 1; s >>= 1) {
    const unsigned long long o = __shfl_xor(x, s);
    x = o < x ? o : x;
  }
  return x;
}

// k rounds, each the smallest rank word above the previous winner: the k
// best in order, with no scratch memory.
__global__ void __launch_bounds__(kTopThreads) k_select_top(int B, const float* __restrict__ key, int higher, int k,
                                                             int M, const float* __restrict__ metrics,
                                                             int* __restrict__ top, float* __restrict__ mean) {
  __shared__ unsigned long long part[kTopThreads / kWave];
  __shared__ int chosen[kMaxTop];
  const int tid = static_cast<int>(threadIdx.x);
  unsigned long long last = 0ull;  // below every rank word (the smallest has a non-zero high half)
  for (int j = 0; j < k; ++j) {
    unsigned long long m = ~0ull;
    for (int i = tid; i < B; i += kTopThreads) {
      const unsigned long long w = rank_word(key, i, higher != 0);
      if (w > last && w < m) m = w;
    }
    m = wave_min64(m);
    if ((tid & (kWave - 1)) == 0) part[tid / kWave] = m;
    __syncthreads();
    unsigned long long best = part[0];
    for (int w = 1; w < kTopThreads / kWave; ++w) best = part[w] < best ? part[w] : best;
    last = best;
    // k <= B leaves a word for every round; the clamp only keeps the index valid
    if (tid == 0) chosen[j] = best == ~0ull ? 0 : static_cast<int>(best & 0xFFFFFFFFull);
    __syncthreads();
  }
  for (int j = tid; j < k; j += kTopThreads) top[j] = chosen[j];
  for (int m = tid; m < M; m += kTopThreads) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += static_cast<double>(metrics[static_cast<size_t>(chosen[j]) * M + m]);
    mean[m] = static_cast<float>(s / k);
  }
}

}  // namespace

hipError_t launch_evaluate(const HandView& H, const SdfView& S, const EvalView& E, const EvalConsts& c, int B,
                           const float* q, float* out, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const dim3 grid((B + kCpw - 1) / kCpw), block(kEvalWaves * kWave);
  if (S.layout == kLayoutZPairs)
    hipLaunchKernelGGL(k_evaluate<kLayoutZPairs>, grid, block, 0, stream, H, S, E, c, B, q, out);
  else
    hipLaunchKernelGGL(k_evaluate<kLayoutYZQuads>, grid, block, 0, stream, H, S, E, c, B, q, out);
  return hipGetLastError();
}

hipError_t launch_evaluate_mesh(const HandView& H, const MeshView& M, const EvalView& E, const EvalConsts& c,
                                float bulge, int B, const float* q, float* out, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_evaluate_mesh, dim3(B), dim3(kEvalWaves * kWave), 0, stream, H, M, E, c, bulge, B, q, out);
  return hipGetLastError();
}

hipError_t launch_select_top(int B, const float* key, int higher_is_better, int k, int M, const float* metrics,
                             int* top, float* mean, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_top, dim3(1), dim3(kTopThreads), 0, stream, B, key, higher_is_better, k, M, metrics,
                     top, mean);
  return hipGetLastError();
}

}  // namespace grasp
