// Device-side building blocks shared by the fused and the plain grasp-step
// kernels: wavefront reductions, small vector algebra, the SDF grid sample
// with its second derivative, and the object-rotation exponential with its
// vector-Jacobian product.
#pragma once

#include "internal.h"

// Every multiply-add that is fused is written as fmaf: the arithmetic of a
// candidate is then the same in every tile variant and launch form, so a
// candidate's result does not depend on how it was scheduled.
#pragma clang fp contract(off)

namespace grasp {
namespace dev {

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Butterfly sum over the 64 lanes: pairwise within quads, then mirrored
// half-rows and rows (DPP), then across rows. Every lane ends with the
// same bits (each step adds a value and its partner's, which commute).
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141>(x);  // row_half_mirror
  x += dpp_f<0x140>(x);  // row_mirror
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  return x;
}

// Makes this wave's earlier LDS writes visible to its later LDS reads from
// other lanes, and keeps the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x))};
}
// s a + b
__device__ __forceinline__ V3 axpy(float s, V3 a, V3 b) { return {fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)}; }
// y = M x and y = M^T x for a row-major 3x3 M
__device__ __forceinline__ V3 mul(const float* M, V3 v) {
  return {fmaf(M[0], v.x, fmaf(M[1], v.y, M[2] * v.z)), fmaf(M[3], v.x, fmaf(M[4], v.y, M[5] * v.z)),
          fmaf(M[6], v.x, fmaf(M[7], v.y, M[8] * v.z))};
}
__device__ __forceinline__ V3 mul_t(const float* M, V3 v) {
  return {fmaf(M[0], v.x, fmaf(M[3], v.y, M[6] * v.z)), fmaf(M[1], v.x, fmaf(M[4], v.y, M[7] * v.z)),
          fmaf(M[2], v.x, fmaf(M[5], v.y, M[8] * v.z))};
}
// hardware reciprocal and reciprocal square root (about 1 ulp)
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------------------
// SDF sample: trilinear value and analytic gradient of the vertex-centred
// grid; outside the box, the clamped sample plus the distance to the box.
// ---------------------------------------------------------------------------
struct Sample {
  float phi;
  V3 n;          // gradient of phi in the object frame
  // kept for the second derivative (penetrating samples in the adjoint)
  float dx00, dx10, dx01, dx11;    // x-differences of the 4 corner rows
  float dyx0, dyx1;                 // (v011-v001)-(v010-v000), (v111-v101)-(v110-v100)
  float fx, fy, fz;
  V3 e;          // offset from the clamped point (0 inside)
  float inv_ne;  // 1/|e| (0 inside)
  bool clx, cly, clz;
};

// Grid coordinate of r along one axis: u = (r - lo) / h, its clamp b to
// [0, N-1] and the cell's lower vertex index, as a float, min(floor(b), N-2).
// u stays a rounded product: contracting it into the clamp residual of the
// outside term would turn an interior point's exact zero into a residue.
struct Axis {
  float u, b, i;
};

__device__ __forceinline__ Axis grid_axis(float r, float lo, const SdfView& S) {
  Axis a;
  a.u = __fmul_rn(r - lo, S.inv_h);
  a.b = __builtin_amdgcn_fmed3f(a.u, 0.0f, static_cast<float>(S.n - 1));
  a.i = fminf(floorf(a.b), static_cast<float>(S.n - 2));
  return a;
}

// A sample point located in the grid: the byte offset, in the gather copy of
// layout LAY, of its cell's data (the yz-quad or the z-pair of its lower
// corner; at most 512 * 511^2 * 16 bytes, below 2^31), its
// position in the cell, and its offset from the clamped point in cells
// (exactly 0 on axes where it lies inside the grid box). Computed once when
// the corners are requested and kept until they arrive.
struct Located {
  uint32_t byte;
  float fx, fy, fz;
  float ox, oy, oz;
};

template <int LAY>
__device__ __forceinline__ Located locate(const SdfView& S, V3 r) {
  const Axis ax = grid_axis(r.x, S.lo[0], S), ay = grid_axis(r.y, S.lo[1], S), az = grid_axis(r.z, S.lo[2], S);
  const uint32_t ix = static_cast<uint32_t>(ax.i), iy = static_cast<uint32_t>(ay.i), iz = static_cast<uint32_t>(az.i);
  Located L;
  if constexpr (LAY == kLayoutYZQuads) {
    const uint32_t n = static_cast<uint32_t>(S.n);
    L.byte = ((iz * (n - 1u) + iy) * n + ix) * 16u;
  } else {
    const uint32_t n = static_cast<uint32_t>(S.n);
    L.byte = ((iz * n + iy) * n + ix) * 8u;
  }
  L.fx = ax.b - ax.i;
  L.fy = ay.b - ay.i;
  L.fz = az.b - az.i;
  L.ox = ax.u - ax.b;
  L.oy = ay.u - ay.b;
  L.oz = az.u - az.b;
  return L;
}

// The cell's 8 corners: lo4 = (000, 100, 010, 110), hi4 = (001, 101, 011, 111)
// (32-bit buffer offsets; an offset past cells_bytes reads zeros, never faults).
// yz-quads: two 16-byte loads, vertices i and i + 1 of one row. Z-pairs: two
// 8-byte loads in row (j, k) and two in row (j + 1, k).
template <int LAY>
__device__ __forceinline__ void sdf_corners(const SdfView& S, uint32_t off, float4& lo4, float4& hi4) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(S.cells), static_cast<short>(0),
                                        static_cast<int>(S.cells_bytes), 0x00020000);
  if constexpr (LAY == kLayoutYZQuads) {
    // quads of vertices i and i + 1: (v000, v010, v001, v011), (v100, v110, v101, v111)
    const float4 e0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(off), 0, 0));
    const float4 e1 =
        __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(off + 16u), 0, 0));
    lo4 = make_float4(e0.x, e1.x, e0.y, e1.y);
    hi4 = make_float4(e0.z, e1.z, e0.w, e1.w);
  } else {
    const uint32_t row = static_cast<uint32_t>(S.n) * 8u;
    const float2 a0 = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off), 0, 0));
    const float2 a1 =
        __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off + 8u), 0, 0));
    const float2 b0 =
        __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off + row), 0, 0));
    const float2 b1 =
        __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off + row + 8u), 0, 0));
    lo4 = make_float4(a0.x, a1.x, b0.x, b1.x);
    hi4 = make_float4(a0.y, a1.y, b0.y, b1.y);
  }
}

// Trilinear value and analytic gradient of the located sample from its
// cell's corners.
__device__ __forceinline__ void sample_sdf_from(const SdfView& S, const Located& L, float4 lo4, float4 hi4,
                                                Sample& s) {
  s.fx = L.fx;
  s.fy = L.fy;
  s.fz = L.fz;
  s.dx00 = lo4.y - lo4.x;
  s.dx10 = lo4.w - lo4.z;
  s.dx01 = hi4.y - hi4.x;
  s.dx11 = hi4.w - hi4.z;
  const float c00 = fmaf(s.fx, s.dx00, lo4.x);
  const float c10 = fmaf(s.fx, s.dx10, lo4.z);
  const float c01 = fmaf(s.fx, s.dx01, hi4.x);
  const float c11 = fmaf(s.fx, s.dx11, hi4.z);
  const float dy0 = c10 - c00, dy1 = c11 - c01;
  const float c0 = fmaf(s.fy, dy0, c00), c1 = fmaf(s.fy, dy1, c01);
  const float gz = c1 - c0;
  const float gy = fmaf(s.fz, dy1 - dy0, dy0);
  const float gx0 = fmaf(s.fy, s.dx10 - s.dx00, s.dx00);
  const float gx1 = fmaf(s.fy, s.dx11 - s.dx01, s.dx01);
  const float gx = fmaf(s.fz, gx1 - gx0, gx0);
  s.dyx0 = (hi4.z - hi4.x) - (lo4.z - lo4.x);
  s.dyx1 = (hi4.w - hi4.y) - (lo4.w - lo4.y);
  s.clx = L.ox != 0.0f;
  s.cly = L.oy != 0.0f;
  s.clz = L.oz != 0.0f;
  s.phi = fmaf(s.fz, gz, c0);
  s.n = v3(s.clx ? 0.0f : gx * S.inv_h, s.cly ? 0.0f : gy * S.inv_h, s.clz ? 0.0f : gz * S.inv_h);
  // offset from the clamped point, exactly 0 on unclamped axes
  s.e = v3(L.ox * S.h, L.oy * S.h, L.oz * S.h);
  // outside the box: add the distance to the clamped point and its direction.
  // Inside, |e|^2 = 0 and the finite 1/|e| bound below adds exact zeros, so
  // the sample needs no select (a -0 component becomes +0).
  const float ee = dot(s.e, s.e);
  const float ine = rsq(fmaxf(ee, 1.17549435e-38f));
  s.inv_ne = ee > 0.0f ? ine : 0.0f;
  s.phi = s.phi + ee * ine;
  s.n = axpy(ine, s.e, s.n);
}

__device__ __forceinline__ void sample_sdf(const SdfView& S, V3 r, Sample& s) {
  float4 lo4, hi4;
  if (S.layout == kLayoutZPairs) {
    const Located L = locate<kLayoutZPairs>(S, r);
    sdf_corners<kLayoutZPairs>(S, L.byte, lo4, hi4);
    sample_sdf_from(S, L, lo4, hi4, s);
  } else {
    const Located L = locate<kLayoutYZQuads>(S, r);
    sdf_corners<kLayoutYZQuads>(S, L.byte, lo4, hi4);
    sample_sdf_from(S, L, lo4, hi4, s);
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin (block i to XCD i mod
// 8). This maps them so that each XCD works on one contiguous range of work
// items, and with a locality order on candidates whose contacts touch
// neighbouring grid cells: each XCD's L2 then holds a compact part of the
// grid. A bijection on [0, nblk) for the first nblk blocks (those holding
// work); blocks past nblk keep their index. Results never depend on it.
__device__ __forceinline__ int xcd_block(int nblk) {
  const int blk = static_cast<int>(blockIdx.x);
  if (blk >= nblk) return blk;
  const int per = nblk >> 3, rem = nblk & 7, x = blk & 7;
  return x * per + min(x, rem) + (blk >> 3);
}

// A byte offset past every gather copy (at most 512 * 511^2 * 16 < 0x7F900000
// bytes, plus a row): loads there read zeros and make no memory request, so a
// lane that needs no sample can still issue its gather unconditionally.
constexpr uint32_t kNoCell = 0x7FFF0000u;

// Lower bounds for culling. The block table holds, for every block of 4^3
// cells, the minimum over the grid vertices of the block widened by one cell
// on every side. A trilinear value is at least the minimum of its cell's
// corners, and the sample adds the distance to the grid box outside it; the
// margins (relative 1e-6 on distances, absolute 1e-6 on the sum) lie far above
// the FP32 rounding of the sample, so a bound above t means the sample's value
// exceeds t exactly as the sample computes it (for t = r_dil: d > 0, no
// active constraint, lambda = 0).
__device__ __forceinline__ float bound_at(const SdfView& S, V3 r, float& e) {
  const Axis ax = grid_axis(r.x, S.lo[0], S), ay = grid_axis(r.y, S.lo[1], S), az = grid_axis(r.z, S.lo[2], S);
  const int bx = static_cast<int>(ax.i) >> kBlockShift;
  const int by = static_cast<int>(ay.i) >> kBlockShift;
  const int bz = static_cast<int>(az.i) >> kBlockShift;
  // max-norm distance to the grid box (at most the Euclidean one the sample adds)
  e = fmaxf(fabsf(ax.u - ax.b), fmaxf(fabsf(ay.u - ay.b), fabsf(az.u - az.b))) * S.h;
  return S.bmin[(bz * S.nb + by) * S.nb + bx];
}

// One sample at grid-frame point r: provably above t.
__device__ __forceinline__ bool provably_clear(const SdfView& S, V3 r, float t) {
  float e;
  const float bm = bound_at(S, r, e);
  return fmaf(0.999999f, e, bm - t) > 1e-6f;
}

// H v with H = d(grad phi)/dr of the sample: mixed partials of the trilinear
// blend on unclamped axes, plus (I - e e^T/|e|^2)/|e| on clamped axes.
__device__ __forceinline__ V3 hess_mul(const SdfView& S, const Sample& s, V3 v) {
  const float ih2 = S.inv_h * S.inv_h;
  float hxy = fmaf(s.fz, (s.dx11 - s.dx01) - (s.dx10 - s.dx00), s.dx10 - s.dx00) * ih2;
  float hxz = fmaf(s.fy, (s.dx11 - s.dx10) - (s.dx01 - s.dx00), s.dx01 - s.dx00) * ih2;
  float hyz = fmaf(s.fx, s.dyx1 - s.dyx0, s.dyx0) * ih2;
  if (s.clx || s.cly) hxy = 0.0f;
  if (s.clx || s.clz) hxz = 0.0f;
  if (s.cly || s.clz) hyz = 0.0f;
  V3 out = v3(fmaf(hxy, v.y, hxz * v.z), fmaf(hxy, v.x, hyz * v.z), fmaf(hxz, v.x, hyz * v.y));
  if (s.inv_ne > 0.0f) {
    const V3 eh = s.inv_ne * s.e;
    const float ev = dot(eh, v);
    out.x += s.clx ? fmaf(-eh.x, ev, v.x) * s.inv_ne : 0.0f;
    out.y += s.cly ? fmaf(-eh.y, ev, v.y) * s.inv_ne : 0.0f;
    out.z += s.clz ? fmaf(-eh.z, ev, v.z) * s.inv_ne : 0.0f;
  }
  return out;
}

// ---------------------------------------------------------------------------
// object orientation: R(theta) = I + A [t]x + B [t]x^2 and the derivatives
// A' = dA/ds, B' = dB/ds with s = |t|^2; power series below |t| = 0.5
// ---------------------------------------------------------------------------
struct Rot {
  float R[9];
  V3 th;
  float A, B, Ap, Bp;
};

__device__ __forceinline__ void make_rot(V3 th, Rot& o) {
  const float s = dot(th, th);
  if (s < 0.25f) {
    o.A = 1.0f + s * (-1.0f / 6 + s * (1.0f / 120 + s * (-1.0f / 5040 + s * (1.0f / 362880))));
    o.B = 0.5f + s * (-1.0f / 24 + s * (1.0f / 720 + s * (-1.0f / 40320 + s * (1.0f / 3628800))));
    o.Ap = -1.0f / 6 + s * (1.0f / 60 + s * (-1.0f / 1680 + s * (1.0f / 90720)));
    o.Bp = -1.0f / 24 + s * (1.0f / 360 + s * (-1.0f / 13440 + s * (1.0f / 907200)));
  } else {
    const float t = sqrtf(s);
    float sn, cs;
    sincosf(t, &sn, &cs);
    o.A = sn / t;
    o.B = (1.0f - cs) / s;
    o.Ap = (t * cs - sn) / (2.0f * s * t);
    o.Bp = (t * sn - 2.0f * (1.0f - cs)) / (2.0f * s * s);
  }
  o.th = th;
  const float x = th.x, y = th.y, z = th.z;
  // [t]x^2 = t t^T - s I
  o.R[0] = 1.0f + o.B * (x * x - s);
  o.R[1] = -o.A * z + o.B * x * y;
  o.R[2] = o.A * y + o.B * x * z;
  o.R[3] = o.A * z + o.B * x * y;
  o.R[4] = 1.0f + o.B * (y * y - s);
  o.R[5] = -o.A * x + o.B * y * z;
  o.R[6] = -o.A * y + o.B * x * z;
  o.R[7] = o.A * x + o.B * y * z;
  o.R[8] = 1.0f + o.B * (z * z - s);
}

// d/dphi of y = R(phi) v contracted with yb, at phi = sgn * theta.
__device__ __forceinline__ V3 rot_vjp(const Rot& o, float sgn, V3 v, V3 yb) {
  const V3 ph = sgn * o.th;
  const V3 tv = cross(ph, v);
  const V3 ttv = cross(ph, tv);
  const float c = 2.0f * o.Ap * dot(yb, tv) + 2.0f * o.Bp * dot(yb, ttv);
  const V3 a = cross(v, yb);
  const float pv = dot(ph, v), py = dot(ph, yb), vy = dot(v, yb);
  return v3(c * ph.x + o.A * a.x + o.B * (pv * yb.x + v.x * py - 2.0f * ph.x * vy),
            c * ph.y + o.A * a.y + o.B * (pv * yb.y + v.y * py - 2.0f * ph.y * vy),
            c * ph.z + o.A * a.z + o.B * (pv * yb.z + v.z * py - 2.0f * ph.z * vy));
}

// Coulomb friction of an active contact (read as positional friction of
// position-based dynamics): the object's material point at the contact moved
// by dp over the step; its tangential part dp_t = dp - (dp . n) n, n = g/|g|,
// is removed up to mu C, as the Eq. (1) correction of a positional
// constraint along t = dp_t / |dp_t|: lambda_t = -min(|dp_t|, mu C) / w_t,
// w_t = |t|^2 + |a x t|^2 / (I/m), correction lambda_t (t, a x t).
struct Fric {
  V3 nh;       // unit normal g / |g|
  float ing;   // 1 / |g|
  float sn;    // dp . n
  V3 th;       // unit tangent of the slide
  float itl;   // 1 / |dp_t|
  float tl;    // |dp_t|
  V3 ut;       // a x t
  float wt;    // generalized inverse mass along t
};

// Contact tolerance: a sample counts as penetrating (an active constraint,
// with the full derivative of C = -d) when d < -kContactTol dt v0. A
// constraint that a projection has just resolved sits at d = 0 up to
// rounding; the tolerance keeps it out of the active set instead of letting
// rounding pick its state, derivative rule and the averaging count. The
// penetration energy at the rest pose counts d < 0 (1/2 d^2 is smooth there).
constexpr float kContactTol = 5e-3f;

// Slides up to this fraction of the test displacement dt v0 have no
// direction and get no friction: a slide that is zero in exact arithmetic (a
// test moving along a flat face's normal) would otherwise take its direction
// from rounding.
constexpr float kSlideMin = 1e-3f;

// The friction direction of a sample with gradient g != 0 (every sample with
// w > w_min has one); false when the slide is no longer than the floor smin.
__device__ __forceinline__ bool friction_dir(V3 g, V3 dp, V3 a, float inv_Im, float smin, Fric& f) {
  f.ing = rsq(dot(g, g));
  f.nh = f.ing * g;
  f.sn = dot(dp, f.nh);
  const V3 dpt = axpy(-f.sn, f.nh, dp);
  const float tl2 = dot(dpt, dpt);
  if (!(tl2 > smin * smin)) return false;
  f.itl = rsq(tl2);
  f.tl = tl2 * f.itl;
  f.th = f.itl * dpt;
  f.ut = cross(a, f.th);
  f.wt = fmaf(dot(f.ut, f.ut), inv_Im, dot(f.th, f.th));
  return true;
}

// Test point of velocity test m before any correction (a = p - dt v0 dir_m):
// exactly one coordinate moves, so the other two (and their grid
// coordinates) are shared by the tests of one contact.
__device__ __forceinline__ V3 test_point(V3 p, int m, float dv) {
  V3 a = p;
  if (m == 0) a.x = p.x - dv;
  else if (m == 1) a.x = p.x + dv;
  else if (m == 2) a.y = p.y - dv;
  else if (m == 3) a.y = p.y + dv;
  else if (m == 4) a.z = p.z - dv;
  else if (m == 5) a.z = p.z + dv;
  return a;
}

__device__ __forceinline__ V3 sim_dir(int m) {
  return v3(m == 0 ? 1.0f : (m == 1 ? -1.0f : 0.0f), m == 2 ? 1.0f : (m == 3 ? -1.0f : 0.0f),
            m == 4 ? 1.0f : (m == 5 ? -1.0f : 0.0f));
}

// Pose of link l for configuration qb (Sec. III-C, p = FK(q)), composed along
// its chain from the wrist: T_0 = Trans(q0..2) Rz(q3) Ry(q4) Rx(q5), then
// T_a = T_parent(a) O_a Rot(axis_a, q_{5+a}) for each link a down to l.
// Writes T (row-major 3x4) and Jw = (world origin, world axis) of joint l
// (for the palm: the wrist origin and a zero axis).
__device__ __forceinline__ void link_transform(const HandView& H, const float* qb, int l, float* T, float* Jw) {
  float R[9], t[3];
  {
    float s3, c3, s4, c4, s5, c5;
    sincosf(qb[3], &s3, &c3);
    sincosf(qb[4], &s4, &c4);
    sincosf(qb[5], &s5, &c5);
    R[0] = c3 * c4; R[1] = fmaf(c3 * s4, s5, -(s3 * c5)); R[2] = fmaf(c3 * s4, c5, s3 * s5);
    R[3] = s3 * c4; R[4] = fmaf(s3 * s4, s5, c3 * c5);    R[5] = fmaf(s3 * s4, c5, -(c3 * s5));
    R[6] = -s4;     R[7] = c4 * s5;                        R[8] = c4 * c5;
    t[0] = qb[0]; t[1] = qb[1]; t[2] = qb[2];
  }
  if (l == 0) {
    Jw[0] = t[0]; Jw[1] = t[1]; Jw[2] = t[2]; Jw[3] = 0.0f; Jw[4] = 0.0f; Jw[5] = 0.0f;
  }
  const int dep = H.depth[l];
  for (int s = 0; s < dep; ++s) {
    const int a = H.chain[l * kMaxDepth + s];
    const float* O = H.origin + 12 * a;
    float JR[9], Jt[3];
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j)
        JR[3 * i + j] = fmaf(R[3 * i], O[j], fmaf(R[3 * i + 1], O[4 + j], R[3 * i + 2] * O[8 + j]));
      Jt[i] = fmaf(R[3 * i], O[3], fmaf(R[3 * i + 1], O[7], fmaf(R[3 * i + 2], O[11], t[i])));
    }
    const V3 k = v3(H.axis[3 * a], H.axis[3 * a + 1], H.axis[3 * a + 2]);
    float sn, cs;
    sincosf(qb[5 + a], &sn, &cs);
    const float oc = 1.0f - cs;
    // Rodrigues: I + sin [k]x + (1 - cos) [k]x^2, with [k]x^2 = k k^T - I
    const float Q[9] = {fmaf(oc, fmaf(k.x, k.x, -1.0f), 1.0f), fmaf(oc, k.x * k.y, -(sn * k.z)),
                        fmaf(oc, k.x * k.z, sn * k.y),         fmaf(oc, k.x * k.y, sn * k.z),
                        fmaf(oc, fmaf(k.y, k.y, -1.0f), 1.0f), fmaf(oc, k.y * k.z, -(sn * k.x)),
                        fmaf(oc, k.x * k.z, -(sn * k.y)),      fmaf(oc, k.y * k.z, sn * k.x),
                        fmaf(oc, fmaf(k.z, k.z, -1.0f), 1.0f)};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        R[3 * i + j] = fmaf(JR[3 * i], Q[j], fmaf(JR[3 * i + 1], Q[3 + j], JR[3 * i + 2] * Q[6 + j]));
    t[0] = Jt[0]; t[1] = Jt[1]; t[2] = Jt[2];
    if (s == dep - 1) {
      const V3 kw = mul(JR, k);
      Jw[0] = Jt[0]; Jw[1] = Jt[1]; Jw[2] = Jt[2]; Jw[3] = kw.x; Jw[4] = kw.y; Jw[5] = kw.z;
    }
  }
  T[0] = R[0]; T[1] = R[1]; T[2] = R[2];  T[3] = t[0];
  T[4] = R[3]; T[5] = R[4]; T[6] = R[5];  T[7] = t[1];
  T[8] = R[6]; T[9] = R[7]; T[10] = R[8]; T[11] = t[2];
}

// World position of a link-local point under a row-major 3x4 transform.
__device__ __forceinline__ V3 xform_point(float4 r0, float4 r1, float4 r2, float lx, float ly, float lz) {
  return v3(fmaf(r0.x, lx, fmaf(r0.y, ly, fmaf(r0.z, lz, r0.w))),
            fmaf(r1.x, lx, fmaf(r1.y, ly, fmaf(r1.z, lz, r1.w))),
            fmaf(r2.x, lx, fmaf(r2.y, ly, fmaf(r2.z, lz, r2.w))));
}

// Gradient of the loss w.r.t. joint j from the subtree wrench (f, tau about
// the world origin) of the link it drives: revolute joints turn about their
// world axis through their world origin o, tau_o = tau - o x f. Wrist joints
// 0..2 translate; 3..5 turn about z, Rz y and Rz Ry x through the wrist origin.
__device__ __forceinline__ float joint_torque(int j, const float* qb, V3 f, V3 tau, V3 o, V3 ax) {
  if (j < 3) return j == 0 ? f.x : (j == 1 ? f.y : f.z);
  const V3 tq = tau - cross(o, f);
  if (j >= 6) return dot(ax, tq);
  float s3, c3, s4, c4;
  sincosf(qb[3], &s3, &c3);
  sincosf(qb[4], &s4, &c4);
  V3 w;
  if (j == 3) w = v3(0.0f, 0.0f, 1.0f);
  else if (j == 4) w = v3(-s3, c3, 0.0f);
  else w = v3(c3 * c4, s3 * c4, -s4);
  return dot(w, tq);
}

}  // namespace dev
}  // namespace grasp
