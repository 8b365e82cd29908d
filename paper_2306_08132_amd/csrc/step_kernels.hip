// gfx950 kernels of the grid-SDF grasp step (Fast-Grasp'D, Sec. III-C and
// Sec. IV-A): forward kinematics, SDF gathers, PBD constraint corrections
// (Eq. (1)) summed per velocity test, stability/penetration/joint losses,
// the hand-written adjoint with the leaky contact gradient, and Adam.
//
// Execution model: one 64-lane wavefront owns one candidate grasp from start
// to end. Lanes stride over the link-sorted contacts in 64-contact chunks;
// every per-candidate reduction (the 7 x 6 correction sums, link wrenches,
// losses) is a wavefront reduction in a fixed order, so a candidate's result
// is bit-identical whatever else runs on the GPU. No workgroup barrier is
// used: waves never wait on each other.
#include "internal.h"

namespace grasp {

namespace {

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
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// y = M x and y = M^T x for a row-major 3x3 M
__device__ __forceinline__ V3 mul(const float* M, V3 v) {
  return {M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
          M[6] * v.x + M[7] * v.y + M[8] * v.z};
}
__device__ __forceinline__ V3 mul_t(const float* M, V3 v) {
  return {M[0] * v.x + M[3] * v.y + M[6] * v.z, M[1] * v.x + M[4] * v.y + M[7] * v.z,
          M[2] * v.x + M[5] * v.y + M[8] * v.z};
}

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

__device__ __forceinline__ void sample_sdf(const SdfView& S, V3 r, Sample& s) {
  const float top = static_cast<float>(S.n - 1);
  // u stays a rounded product: contracting it into the clamp residual below
  // would turn an interior point's exact zero offset into a rounding residue
  const float ux = __fmul_rn(r.x - S.lo[0], S.inv_h);
  const float uy = __fmul_rn(r.y - S.lo[1], S.inv_h);
  const float uz = __fmul_rn(r.z - S.lo[2], S.inv_h);
  const float bx = fminf(fmaxf(ux, 0.0f), top);
  const float by = fminf(fmaxf(uy, 0.0f), top);
  const float bz = fminf(fmaxf(uz, 0.0f), top);
  const int cm = S.n - 2;
  const int ix = min(max(static_cast<int>(floorf(bx)), 0), cm);
  const int iy = min(max(static_cast<int>(floorf(by)), 0), cm);
  const int iz = min(max(static_cast<int>(floorf(bz)), 0), cm);
  s.fx = bx - static_cast<float>(ix);
  s.fy = by - static_cast<float>(iy);
  s.fz = bz - static_cast<float>(iz);
  const int nc = S.n - 1;
  const int cell = (iz * nc + iy) * nc + ix;
  const float4 lo4 = S.cells[2 * cell];
  const float4 hi4 = S.cells[2 * cell + 1];
  // corners: lo4 = (000, 100, 010, 110), hi4 = (001, 101, 011, 111)
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
  s.clx = ux != bx;
  s.cly = uy != by;
  s.clz = uz != bz;
  s.phi = fmaf(s.fz, gz, c0);
  s.n = v3(s.clx ? 0.0f : gx * S.inv_h, s.cly ? 0.0f : gy * S.inv_h, s.clz ? 0.0f : gz * S.inv_h);
  s.e = v3(s.clx ? (ux - bx) * S.h : 0.0f, s.cly ? (uy - by) * S.h : 0.0f, s.clz ? (uz - bz) * S.h : 0.0f);
  const float ee = dot(s.e, s.e);
  s.inv_ne = 0.0f;
  if (ee > 0.0f) {
    const float ne = sqrtf(ee);
    s.inv_ne = 1.0f / ne;
    s.phi += ne;
    s.n = s.n + s.inv_ne * s.e;
  }
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
  V3 out = v3(hxy * v.y + hxz * v.z, hxy * v.x + hyz * v.z, hxz * v.x + hyz * v.y);
  if (s.inv_ne > 0.0f) {
    const V3 eh = s.inv_ne * s.e;
    const float ev = dot(eh, v);
    out.x += s.clx ? (v.x - eh.x * ev) * s.inv_ne : 0.0f;
    out.y += s.cly ? (v.y - eh.y * ev) * s.inv_ne : 0.0f;
    out.z += s.clz ? (v.z - eh.z * ev) * s.inv_ne : 0.0f;
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

__device__ __forceinline__ V3 sim_dir(int m) {
  return v3(m == 0 ? 1.0f : (m == 1 ? -1.0f : 0.0f), m == 2 ? 1.0f : (m == 3 ? -1.0f : 0.0f),
            m == 4 ? 1.0f : (m == 5 ? -1.0f : 0.0f));
}

// ---------------------------------------------------------------------------
// per-wave LDS layout (floats)
// ---------------------------------------------------------------------------
constexpr int kOffT = 0;                                // [kMaxLinks][12] link transforms
constexpr int kOffJ = kOffT + kMaxLinks * 12;           // [kMaxLinks][6] joint origin, world axis
constexpr int kOffW = kOffJ + kMaxLinks * 6;            // [kMaxLinks][6] link force, torque (adjoint)
constexpr int kOffU = kOffW + kMaxLinks * 6;            // [7][32] per-test pose constants
constexpr int kOffPose = kOffU + kSims * 32;            // [slots][7][6] pose checkpoints
constexpr int kUStride = 32;
// per-test constants: 0..2 x, 3..11 R, 12..14 theta, 15..18 A B A' B', 19..24 Wl_bar Wa_bar

struct Ctx {
  const HandView& H;
  const SdfView& S;
  const StepConsts& P;
  float* lds;
  int lane;
};

// Link transforms T_l (Sec. III-C, p = FK(q)). Each lane l composes its own
// chain from the wrist: T_0 = Trans(q0..2) Rz(q3) Ry(q4) Rx(q5), then
// T_a = T_parent(a) O_a Rot(axis_a, q_{5+a}) down to link l. Also stores each
// joint's world origin and world axis for the adjoint.
__device__ void forward_kinematics(const Ctx& c, const float* qb) {
  const HandView& H = c.H;
  const int l = c.lane;
  float R[9], t[3];
  {
    float s3, c3, s4, c4, s5, c5;
    sincosf(qb[3], &s3, &c3);
    sincosf(qb[4], &s4, &c4);
    sincosf(qb[5], &s5, &c5);
    R[0] = c3 * c4; R[1] = c3 * s4 * s5 - s3 * c5; R[2] = c3 * s4 * c5 + s3 * s5;
    R[3] = s3 * c4; R[4] = s3 * s4 * s5 + c3 * c5; R[5] = s3 * s4 * c5 - c3 * s5;
    R[6] = -s4;     R[7] = c4 * s5;                R[8] = c4 * c5;
    t[0] = qb[0]; t[1] = qb[1]; t[2] = qb[2];
  }
  if (l < H.L) {
    float* Jw = c.lds + kOffJ + 6 * l;
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
          JR[3 * i + j] = R[3 * i] * O[j] + R[3 * i + 1] * O[4 + j] + R[3 * i + 2] * O[8 + j];
        Jt[i] = R[3 * i] * O[3] + R[3 * i + 1] * O[7] + R[3 * i + 2] * O[11] + t[i];
      }
      const V3 k = v3(H.axis[3 * a], H.axis[3 * a + 1], H.axis[3 * a + 2]);
      float sn, cs;
      sincosf(qb[5 + a], &sn, &cs);
      const float oc = 1.0f - cs;
      // Rodrigues: I + sin [k]x + (1 - cos) [k]x^2, [k]x^2 = k k^T - I
      const float Q[9] = {1.0f + oc * (k.x * k.x - 1.0f), -sn * k.z + oc * k.x * k.y, sn * k.y + oc * k.x * k.z,
                          sn * k.z + oc * k.x * k.y, 1.0f + oc * (k.y * k.y - 1.0f), -sn * k.x + oc * k.y * k.z,
                          -sn * k.y + oc * k.x * k.z, sn * k.x + oc * k.y * k.z, 1.0f + oc * (k.z * k.z - 1.0f)};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          R[3 * i + j] = JR[3 * i] * Q[j] + JR[3 * i + 1] * Q[3 + j] + JR[3 * i + 2] * Q[6 + j];
      t[0] = Jt[0]; t[1] = Jt[1]; t[2] = Jt[2];
      if (s == dep - 1) {
        const V3 kw = mul(JR, k);
        Jw[0] = Jt[0]; Jw[1] = Jt[1]; Jw[2] = Jt[2]; Jw[3] = kw.x; Jw[4] = kw.y; Jw[5] = kw.z;
      }
    }
    float* T = c.lds + kOffT + 12 * l;
    T[0] = R[0]; T[1] = R[1]; T[2] = R[2]; T[3] = t[0];
    T[4] = R[3]; T[5] = R[4]; T[6] = R[5]; T[7] = t[1];
    T[8] = R[6]; T[9] = R[7]; T[10] = R[8]; T[11] = t[2];
  }
  wave_lds_sync();
}

// Contact i of chunk ch for this lane: world position p (0 for padding).
__device__ __forceinline__ V3 contact_point(const Ctx& c, int i, int& link) {
  const HandView& H = c.H;
  const float lx = H.cx[i], ly = H.cy[i], lz = H.cz[i];
  link = H.clink[i];
  const float4* T4 = reinterpret_cast<const float4*>(c.lds + kOffT + 12 * link);
  const float4 r0 = T4[0], r1 = T4[1], r2 = T4[2];
  return v3(fmaf(r0.x, lx, fmaf(r0.y, ly, fmaf(r0.z, lz, r0.w))),
            fmaf(r1.x, lx, fmaf(r1.y, ly, fmaf(r1.z, lz, r1.w))),
            fmaf(r2.x, lx, fmaf(r2.y, ly, fmaf(r2.z, lz, r2.w))));
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

// One forward projection iteration over all contacts: the 7 x 6 correction
// sums W_m = sum_i lambda_i (g_i, u_i) (Eq. (1) per constraint, summed) and,
// on the rest test of the first iteration, the penetration energy.
template <bool KONE>
__device__ void forward_pass(const Ctx& c, bool first, float W[kSims][6], float& lpen,
                             float* trace_s /*caller-order samples for this k, or null*/,
                             int K, int k) {
  const HandView& H = c.H;
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, dv = c.P.dt * c.P.v0;
  for (int m = 0; m < kSims; ++m)
    for (int j = 0; j < 6; ++j) W[m][j] = 0.0f;
  lpen = 0.0f;
  for (int ch = 0; ch < H.n_chunks; ++ch) {
    const int i = ch * kWave + c.lane;
    const bool valid = i < H.Nc;
    int link;
    const V3 p = contact_point(c, i, link);
#pragma unroll
    for (int m = 0; m < kSims; ++m) {
      V3 a, r;
      Rot o;
      if constexpr (KONE) {
        a = p - dv * sim_dir(m);
        r = a;
      } else {
        const float* U = c.lds + kOffU + kUStride * m;
        load_rot(U, o);
        a = p - v3(U[0], U[1], U[2]);
        r = mul_t(o.R, a);
      }
      Sample s;
      sample_sdf(S, r, s);
      const V3 g = KONE ? s.n : mul(o.R, s.n);
      const float d = s.phi - rd;
      if (first && m == kSims - 1 && valid && d < 0.0f) lpen = fmaf(0.5f * d, d, lpen);
      float lam = 0.0f, w = 0.0f;
      if (valid && (d < 0.0f || trace_s)) {
        const V3 u = cross(a, g);
        w = dot(g, g) + dot(u, u) * S.inv_Im;
        if (d < 0.0f && w > wmin) {
          lam = d / w;
          W[m][0] = fmaf(lam, g.x, W[m][0]);
          W[m][1] = fmaf(lam, g.y, W[m][1]);
          W[m][2] = fmaf(lam, g.z, W[m][2]);
          W[m][3] = fmaf(lam, u.x, W[m][3]);
          W[m][4] = fmaf(lam, u.y, W[m][4]);
          W[m][5] = fmaf(lam, u.z, W[m][5]);
        }
      }
      if (trace_s && valid) {
        float* o6 = trace_s + ((static_cast<size_t>(m) * K + k) * H.Nc + H.perm[i]) * 6;
        o6[0] = d; o6[1] = g.x; o6[2] = g.y; o6[3] = g.z; o6[4] = w; o6[5] = lam;
      }
    }
  }
  for (int m = 0; m < kSims; ++m)
    for (int j = 0; j < 6; ++j) W[m][j] = wave_sum(W[m][j]);
  lpen = wave_sum(lpen);
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

// One backward iteration over all contacts (the adjoint of forward_pass at
// iteration k). The per-test seeds Wl_bar, Wa_bar (adjoints of the summed
// corrections) are in LDS. Adds p_bar x p and p_bar to the link wrench table
// and, when pose_adj, returns the pose adjoint sums (-sum a_bar, sum theta_bar).
template <bool KONE>
__device__ void backward_pass(const Ctx& c, bool first, float pen_seed, bool pose_adj,
                              float XB[kSims][6]) {
  const HandView& H = c.H;
  const SdfView& S = c.S;
  const float rd = c.P.r_dil, wmin = c.P.w_min, alpha = c.P.alpha, dv = c.P.dt * c.P.v0;
  const float inv_Im = S.inv_Im;
  if (pose_adj)
    for (int m = 0; m < kSims; ++m)
      for (int j = 0; j < 6; ++j) XB[m][j] = 0.0f;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  int cur = -1;
  for (int ch = 0; ch < H.n_chunks; ++ch) {
    const int i = ch * kWave + c.lane;
    const bool valid = i < H.Nc;
    int link;
    const V3 p = contact_point(c, i, link);
    V3 pbar = v3(0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int m = 0; m < kSims; ++m) {
      const float* U = c.lds + kOffU + kUStride * m;
      V3 a, r;
      Rot o;
      if constexpr (KONE) {
        a = p - dv * sim_dir(m);
        r = a;
      } else {
        load_rot(U, o);
        a = p - v3(U[0], U[1], U[2]);
        r = mul_t(o.R, a);
      }
      Sample s;
      sample_sdf(S, r, s);
      const V3 g = KONE ? s.n : mul(o.R, s.n);
      const float d = s.phi - rd;
      const V3 u = cross(a, g);
      const float w = dot(g, g) + dot(u, u) * inv_Im;
      const V3 WlB = v3(U[19], U[20], U[21]);
      const V3 WaB = v3(U[22], U[23], U[24]);
      const float lb = dot(WlB, g) + dot(WaB, u);
      float dbar = 0.0f;
      V3 gbar = v3(0.0f, 0.0f, 0.0f), abar = v3(0.0f, 0.0f, 0.0f);
      bool pen = false;
      if (valid && w > wmin) {
        const float iw = 1.0f / w;
        if (d < 0.0f) {
          // lambda = d / w: full derivative through d, g and u
          pen = true;
          const float lam = d * iw;
          dbar = lb * iw;
          const float wbar2 = -2.0f * lb * lam * iw;
          V3 ubar = lam * WaB + (wbar2 * inv_Im) * u;
          gbar = lam * WlB + wbar2 * g;
          abar = cross(g, ubar);
          gbar = gbar + cross(ubar, a);
        } else {
          // leaky rule: dC/dd = -alpha where the point does not penetrate
          dbar = alpha * lb * iw;
        }
      }
      if (first && m == kSims - 1 && valid && d < 0.0f) dbar = fmaf(pen_seed, d, dbar);
      V3 rbar;
      if constexpr (KONE) {
        rbar = dbar * s.n;
        if (pen) rbar = rbar + hess_mul(S, s, gbar);
        abar = abar + rbar;
      } else {
        const V3 nbar = mul_t(o.R, gbar);
        rbar = dbar * s.n;
        if (pen) rbar = rbar + hess_mul(S, s, nbar);
        abar = abar + mul(o.R, rbar);
        if (pose_adj && valid) {
          V3 thb = v3(0.0f, 0.0f, 0.0f);
          if (pen) thb = rot_vjp(o, 1.0f, s.n, gbar);
          thb = thb - rot_vjp(o, -1.0f, a, rbar);
          XB[m][0] -= abar.x; XB[m][1] -= abar.y; XB[m][2] -= abar.z;
          XB[m][3] += thb.x; XB[m][4] += thb.y; XB[m][5] += thb.z;
        }
      }
      pbar = pbar + abar;
    }
    // scatter p_bar into link wrenches (force, torque about the world origin)
    const V3 tau = cross(p, pbar);
    const float v6[6] = {pbar.x, pbar.y, pbar.z, tau.x, tau.y, tau.z};
    const int lk = H.chunk_lk[ch];
    const int lf = lk & 0xffff, ll = lk >> 16;
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
        for (int j = 0; j < 6; ++j) mv[j] = (link == l && valid) ? v6[j] : 0.0f;
        flush_link(c, l, mv);
      }
    }
  }
  if (cur >= 0) flush_link(c, cur, acc);
  if (pose_adj)
    for (int m = 0; m < kSims; ++m)
      for (int j = 0; j < 6; ++j) XB[m][j] = wave_sum(XB[m][j]);
  wave_lds_sync();
}

__device__ __forceinline__ float* pose_slot(float* lds, int s) { return lds + kOffPose + s * kSims * 6; }

// Writes pose_new = pose_old + (omega W_lin, omega/(I/m) W_ang) for all tests.
__device__ __forceinline__ void advance_pose(const Ctx& c, const float* pold, float* pnew, const float W[kSims][6]) {
  const float om = c.P.omega, omi = c.P.omega * c.S.inv_Im;
  if (c.lane == 0)
    for (int m = 0; m < kSims; ++m)
      for (int j = 0; j < 6; ++j) pnew[6 * m + j] = fmaf(j < 3 ? om : omi, W[m][j], pold[6 * m + j]);
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
template <bool KONE>
__device__ void candidate_step(const StepArgs& A, int b, int kind, bool adam, float* lds) {
  const HandView& H = A.hand;
  const StepConsts& P = A.prm;
  const Ctx c{A.hand, A.sdf, A.prm, lds, lane_id()};
  const int nd = H.n_dof;
  const int lane = c.lane;
  const float* qb = A.q + static_cast<size_t>(b) * nd;
  const float qj = lane < nd ? qb[lane] : 0.0f;
  const int K = P.K, ck = P.ckpt;
  const int nslots = K / ck + 1;
  const bool do_fwd = (kind != STEP_BWD) || A.poses == nullptr;
  const bool do_bwd = kind != STEP_FWD;
  float* gpose = A.poses ? A.poses + static_cast<size_t>(b) * kSims * nslots * 6 : nullptr;

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
  float W[kSims][6];
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
      forward_pass<KONE>(c, k == 0, W, lp, ts, K, k);
      if (k == 0) lpen = lp;
      advance_pose(c, cur, cur, W);
      if ((k + 1) % ck == 0) {
        float* dst = pose_slot(lds, (k + 1) / ck);
        if (lane < kSims * 6) dst[lane] = cur[lane];
        wave_lds_sync();
      }
    }
    if (A.trace_poses && lane < kSims * 6)
      A.trace_poses[((static_cast<size_t>(b) * kSims + lane / 6) * (K + 1) + K) * 6 + lane % 6] = cur[lane];
    if (gpose && kind == STEP_FWD)
      for (int t = lane; t < nslots * kSims * 6; t += kWave) gpose[t] = lds[kOffPose + t];
  } else {
    for (int t = lane; t < nslots * kSims * 6; t += kWave) lds[kOffPose + t] = gpose[t];
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
    const float L = P.w_stable * Lstable + P.w_pen * lpen + P.w_range * Lrange + P.w_limit * Llimit;
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
  // seeds: d L / d x^K_m and d L / d theta^K_m
  float XB[kSims][6];
  {
    const float cst = sL * P.w_stable / (kSims * P.dt);
    for (int m = 0; m < kSims; ++m) {
      const float* pm = fin + 6 * m;
      const V3 x = v3(pm[0], pm[1], pm[2]), th = v3(pm[3], pm[4], pm[5]);
      const float nx = sqrtf(dot(x, x)), nt = sqrtf(dot(th, th));
      // |v| = |x|/dt; its derivative is x/|x| / dt (0 at the origin)
      const float fx = nx > 0.0f ? cst / nx : 0.0f;
      const float ft = nt > 0.0f ? cst / nt : 0.0f;
      XB[m][0] = fx * x.x; XB[m][1] = fx * x.y; XB[m][2] = fx * x.z;
      XB[m][3] = ft * th.x; XB[m][4] = ft * th.y; XB[m][5] = ft * th.z;
    }
  }
  const float pen_seed = sL * P.w_pen;
  const int nseg = K / ck;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    // replay the segment's iterations from its checkpoint (none when ck = 1)
    float* segbuf = pose_slot(lds, nslots);  // ck slots: poses seg*ck .. seg*ck+ck-1
    {
      const float* ckp = pose_slot(lds, seg);
      if (lane < kSims * 6) segbuf[lane] = ckp[lane];
      wave_lds_sync();
      for (int j = 1; j < ck; ++j) {
        if constexpr (!KONE) load_test_consts(c, segbuf + (j - 1) * kSims * 6);
        float lp;
        forward_pass<KONE>(c, false, W, lp, nullptr, K, seg * ck + j - 1);
        advance_pose(c, segbuf + (j - 1) * kSims * 6, segbuf + j * kSims * 6, W);
      }
    }
    for (int j = ck - 1; j >= 0; --j) {
      const int k = seg * ck + j;
      if constexpr (!KONE) load_test_consts(c, segbuf + j * kSims * 6);
      // seeds of this iteration's correction sums
      if (lane < kSims) {
        float* U = lds + kOffU + kUStride * lane;
        const float om = P.omega, omi = P.omega * c.S.inv_Im;
        float xb[6];
        for (int m = 0; m < kSims; ++m)
          if (m == lane)
            for (int t = 0; t < 6; ++t) xb[t] = XB[m][t];
        U[19] = om * xb[0]; U[20] = om * xb[1]; U[21] = om * xb[2];
        U[22] = omi * xb[3]; U[23] = omi * xb[4]; U[24] = omi * xb[5];
      }
      wave_lds_sync();
      float D[kSims][6];
      const bool need_pose = !KONE && k > 0;
      backward_pass<KONE>(c, k == 0, pen_seed, need_pose, D);
      if (need_pose)
        for (int m = 0; m < kSims; ++m)
          for (int t = 0; t < 6; ++t) XB[m][t] += D[m][t];
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
  {
    const float* W0 = lds + kOffW;
    const float* J0 = lds + kOffJ;
    if (lane < 3) {
      gq = W0[lane];
    } else if (lane < 6) {
      // wrist rotations about the axes through the wrist origin t0
      const V3 f = v3(W0[0], W0[1], W0[2]), tau = v3(W0[3], W0[4], W0[5]);
      const V3 t0 = v3(J0[0], J0[1], J0[2]);
      const V3 tq = tau - cross(t0, f);
      float s3, c3, s4, c4;
      sincosf(qb[3], &s3, &c3);
      sincosf(qb[4], &s4, &c4);
      V3 ax;
      if (lane == 3) ax = v3(0.0f, 0.0f, 1.0f);
      else if (lane == 4) ax = v3(-s3, c3, 0.0f);
      else ax = v3(c3 * c4, s3 * c4, -s4);
      gq = dot(ax, tq);
    } else if (lane < nd) {
      const int l = lane - 5;
      const float* Wl = lds + kOffW + 6 * l;
      const float* Jl = lds + kOffJ + 6 * l;
      const V3 f = v3(Wl[0], Wl[1], Wl[2]), tau = v3(Wl[3], Wl[4], Wl[5]);
      const V3 o = v3(Jl[0], Jl[1], Jl[2]), ax = v3(Jl[3], Jl[4], Jl[5]);
      gq = dot(ax, tau - cross(o, f));
      // joint losses
      const float rg = Lrange > 0.0f ? P.w_range * dm / Lrange : 0.0f;
      const float lg = qj > up ? P.w_limit : (qj < lo ? -P.w_limit : 0.0f);
      gq += sL * (rg + lg);
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

template <bool KONE>
__global__ void __launch_bounds__(256) k_step(StepArgs A, int kind, int adam) {
  extern __shared__ float smem[];
  const int wpb = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int b = blockIdx.x * wpb + w;
  if (b >= A.B) return;
  float* lds = smem + static_cast<size_t>(w) * wave_lds_floats(A.prm.K, A.prm.ckpt);
  candidate_step<KONE>(A, b, kind, adam != 0, lds);
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

__global__ void k_build_cells(const float* __restrict__ vals, int n, float4* __restrict__ cells) {
  const int nc = n - 1;
  const long long total = static_cast<long long>(nc) * nc * nc;
  const long long id = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int ix = static_cast<int>(id % nc);
  const int iy = static_cast<int>((id / nc) % nc);
  const int iz = static_cast<int>(id / (static_cast<long long>(nc) * nc));
  auto V = [&](int i, int j, int k) {
    return vals[(static_cast<long long>(iz + k) * n + (iy + j)) * n + (ix + i)];
  };
  cells[2 * id] = make_float4(V(0, 0, 0), V(1, 0, 0), V(0, 1, 0), V(1, 1, 0));
  cells[2 * id + 1] = make_float4(V(0, 0, 1), V(1, 0, 1), V(0, 1, 1), V(1, 1, 1));
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

hipError_t launch_step(const StepArgs& a, StepKind kind, bool adam, int wpb, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  const int blocks = (a.B + wpb - 1) / wpb;
  const size_t lds = wave_lds_floats(a.prm.K, a.prm.ckpt) * wpb * sizeof(float);
  if (a.prm.K == 1)
    hipLaunchKernelGGL(k_step<true>, dim3(blocks), dim3(wpb * kWave), lds, stream, a, static_cast<int>(kind),
                       adam ? 1 : 0);
  else
    hipLaunchKernelGGL(k_step<false>, dim3(blocks), dim3(wpb * kWave), lds, stream, a, static_cast<int>(kind),
                       adam ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adam(int n, float* q, float* m, float* v, const float* g, AdamConsts c, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, stream, n, q, m, v, g, c);
  return hipGetLastError();
}

hipError_t launch_build_cells(const float* values, int n, float4* cells, hipStream_t stream) {
  const long long total = static_cast<long long>(n - 1) * (n - 1) * (n - 1);
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(k_build_cells, dim3(blocks), dim3(256), 0, stream, values, n, cells);
  return hipGetLastError();
}

hipError_t launch_sample_points(const SdfView& s, int n, const float* r, float* out4, float* hess9,
                                hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_points, dim3((n + 255) / 256), dim3(256), 0, stream, s, n, r, out4, hess9);
  return hipGetLastError();
}

}  // namespace grasp
