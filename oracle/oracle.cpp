// FP64 CPU oracle for the grid-SDF Fast-Grasp'D grasp step.
//
// TEST INFRASTRUCTURE ONLY: the plain reference the GPU path is checked
// against. Shares no code with the GPU library. Every step follows the paper's
// order and notation (Fast-Grasp'D, Sec. III-C "Position-based dynamics" and
// Sec. IV-A "Gradient-based grasp optimization"); the grid sampler follows the
// trilinear grid SDF the paper describes for its predecessor (Sec. III-A).
//
// Gradients: forward-mode dual numbers, one tangent per degree of freedom.
// The leaky contact gradient (Sec. III-C, "Leaky gradient") is a derivative
// rule on C = max(0, -d): its tangent is -dd where d < 0 and -alpha dd
// elsewhere, while its value is unchanged.
//
// Readings where the paper is silent (each listed in the design notes):
//  * object representation: dense grid, trilinear value, analytic gradient;
//    outside the box, clamp to the box and add the Euclidean distance to it;
//  * the paper's Gauss-Seidel step over the contact constraints (Sec. III-C)
//    is taken literally with projection = 1: one constraint after another,
//    each at the pose the previous ones left, in link-major order (the paper
//    gives no order); by default (projection = 0) it is replaced by its
//    parallel form with constraint averaging: every
//    correction of Eq. (1) is computed at the same pose and their sum is
//    divided by the number n of active (penetrating, w > w_min) constraints
//    of that test, then added with relaxation omega; K such iterations in one
//    step. One active constraint gives exactly the Gauss-Seidel update; n
//    aligned constraints are resolved once instead of n times. n is piecewise
//    constant in q, so it carries no derivative;
//  * mass matrix: isotropic, mass 1 and inertia I/m; orientation is a
//    rotation vector updated additively; gravity is absent;
//  * the test velocities are +-v0 along each axis plus zero; angular 0;
//  * penetration loss L_pen = 1/2 sum C^2 at the rest pose; L_range over
//    finger joints; L_limit summed over finger joints;
//  * derivatives at kinks (|.| at 0, max at 0, clamp) are 0; at d = 0 the
//    leaky branch is taken.
#include "oracle_api.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int kSims = 7;  // M = 7 simulations (Sec. IV-A)
// friction floor: slides up to this fraction of dt v0 have no direction
constexpr double kSlideMin = 1e-3;
// contact tolerance: penetration beyond this fraction of dt v0 makes a
// constraint active
constexpr double kContactTol = 5e-3;

// ---------------------------------------------------------------------------
// scalars: double, or a dual number carrying N tangents
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { std::fill(d, d + N, 0.0); }
  Dual(double x) : v(x) { std::fill(d, d + N, 0.0); }  // NOLINT: implicit constant
};

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) {
  Dual<N> r; r.v = a * b.v; for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& b, double a) { return a * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v / b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / b; return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator+(double b, const Dual<N>& a) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> inline Dual<N> operator-(double b, const Dual<N>& a) { return -(a - b); }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }

template <int N> inline double val(const Dual<N>& a) { return a.v; }
inline double val(double a) { return a; }

template <int N> inline Dual<N> sqrt_(const Dual<N>& a) {
  Dual<N> r; r.v = std::sqrt(a.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}
inline double sqrt_(double a) { return std::sqrt(a); }
template <int N> inline Dual<N> sin_(const Dual<N>& a) {
  Dual<N> r; r.v = std::sin(a.v); double c = std::cos(a.v);
  for (int i = 0; i < N; ++i) r.d[i] = c * a.d[i];
  return r;
}
inline double sin_(double a) { return std::sin(a); }
template <int N> inline Dual<N> cos_(const Dual<N>& a) {
  Dual<N> r; r.v = std::cos(a.v); double s = std::sin(a.v);
  for (int i = 0; i < N; ++i) r.d[i] = -s * a.d[i];
  return r;
}
inline double cos_(double a) { return std::cos(a); }

// A value with a zero tangent.
template <class S> inline S konst(double x) { return S(x); }

// Euclidean norm, derivative 0 at the origin (a kink).
template <class S> inline S norm3(const S v[3]) {
  S s = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  if (val(s) > 0.0) return sqrt_(s);
  return konst<S>(0.0);
}

// ---------------------------------------------------------------------------
// rigid transforms (row-major 3x3 rotation + translation)
// ---------------------------------------------------------------------------
template <class S>
struct Xf {
  S R[9];
  S t[3];
};

template <class S> Xf<S> identity_xf() {
  Xf<S> x;
  for (int i = 0; i < 9; ++i) x.R[i] = konst<S>((i % 4 == 0) ? 1.0 : 0.0);
  for (int i = 0; i < 3; ++i) x.t[i] = konst<S>(0.0);
  return x;
}

template <class S> Xf<S> compose(const Xf<S>& A, const Xf<S>& B) {
  Xf<S> C;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      C.R[3 * i + j] = A.R[3 * i] * B.R[j] + A.R[3 * i + 1] * B.R[3 + j] + A.R[3 * i + 2] * B.R[6 + j];
    C.t[i] = A.R[3 * i] * B.t[0] + A.R[3 * i + 1] * B.t[1] + A.R[3 * i + 2] * B.t[2] + A.t[i];
  }
  return C;
}

template <class S> void apply_xf(const Xf<S>& A, const double c[3], S out[3]) {
  for (int i = 0; i < 3; ++i)
    out[i] = A.R[3 * i] * c[0] + A.R[3 * i + 1] * c[1] + A.R[3 * i + 2] * c[2] + A.t[i];
}

// Rotation by angle a about a fixed unit axis k: I + sin a [k]x + (1 - cos a) [k]x^2.
template <class S> Xf<S> axis_angle(const double k[3], const S& a) {
  S s = sin_(a), c1 = 1.0 - cos_(a);
  double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  Xf<S> x;
  for (int i = 0; i < 9; ++i) x.R[i] = ((i % 4 == 0) ? 1.0 : 0.0) + s * K[i] + c1 * K2[i];
  for (int i = 0; i < 3; ++i) x.t[i] = konst<S>(0.0);
  return x;
}

template <class S> Xf<S> const_xf(const double* m12) {
  Xf<S> x;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) x.R[3 * i + j] = konst<S>(m12[4 * i + j]);
    x.t[i] = konst<S>(m12[4 * i + 3]);
  }
  return x;
}

// Forward kinematics p = FK(q) (Sec. III-C): the wrist is
// Trans(q0, q1, q2) Rz(q3) Ry(q4) Rx(q5); each further link l hangs from its
// parent through the fixed joint origin O_l and a revolute joint about axis_l
// by angle q_{5+l}: T_l = T_parent O_l Rot(axis_l, q_{5+l}).
template <class S> void forward_kinematics(const ohand& h, const S* q, std::vector<Xf<S>>& T) {
  const int L = h.n_links;
  T.assign(L, identity_xf<S>());
  const double ez[3] = {0, 0, 1}, ey[3] = {0, 1, 0}, ex[3] = {1, 0, 0};
  Xf<S> root = identity_xf<S>();
  for (int i = 0; i < 3; ++i) root.t[i] = q[i];
  root = compose(root, axis_angle(ez, q[3]));
  root = compose(root, axis_angle(ey, q[4]));
  root = compose(root, axis_angle(ex, q[5]));
  T[0] = root;
  for (int l = 1; l < L; ++l) {
    Xf<S> J = compose(T[h.parent[l]], const_xf<S>(h.joint_origin + 12 * l));
    T[l] = compose(J, axis_angle(h.joint_axis + 3 * l, q[5 + l]));
  }
}

// ---------------------------------------------------------------------------
// object SDF sample: value and gradient at a point in the object frame
// ---------------------------------------------------------------------------
struct SampleInfo {
  int cell[3] = {0, 0, 0};
  int clamped[3] = {0, 0, 0};
  double face_margin = 1e30;
  double axis_margin[3] = {1e30, 1e30, 1e30};  // per axis: distance (cell units) to the nearest face
  // input: bit a set = take the cell on the other side of the face nearest
  // to the sample along axis a (both cells meet there: the value is the same,
  // the gradient is the other cell's)
  int flip_axes = 0;
  // mesh: input, take the other side of the flat surface; output, the flat
  // distance (the sign's margin)
  int flip_sign = 0;
  double sign_margin = 1e30;
  // mesh: input, take the nearest different point of the surface; output,
  // how much farther it is (0 on the medial axis)
  int flip_alt = 0;
  double alt_margin = 1e30;
  // mesh: input, take the neighbouring region of the closest point (face
  // interior, edge, vertex); output, its distance to that region
  int flip_region = 0;
  double region_margin = 1e30;
};

// Grid: trilinear interpolation of a vertex-centred grid (Sec. III-A). Per
// axis u = (r - lo)/h, clamped to [0, N-1]; the cell is floor(u) capped at
// N-2 and f = u - cell. The gradient is the analytic derivative of the
// trilinear blend, zero along clamped axes. Outside the box the distance e
// from the clamped point is added to the value and e/|e| to the gradient.
template <class S>
void sample_grid(const oobject& o, const S r[3], S& phi, S n[3], SampleInfo* info) {
  const int N = o.n;
  S f[3];
  S e[3];
  int c[3];
  bool cl[3];
  double margin = 1e30;
  for (int a = 0; a < 3; ++a) {
    S u = (r[a] - o.lo[a]) / o.h;
    S ub;
    if (val(u) < 0.0) { ub = konst<S>(0.0); cl[a] = true; }
    else if (val(u) > N - 1.0) { ub = konst<S>(N - 1.0); cl[a] = true; }
    else { ub = u; cl[a] = false; }
    c[a] = std::min(static_cast<int>(std::floor(val(ub))), N - 2);
    double k = std::min(std::max(std::round(val(u)), 0.0), N - 1.0);
    bool outward = false;  // clamped by the other reading at a boundary face
    if (info && (info->flip_axes >> a & 1)) {
      const int kf = static_cast<int>(k);
      if (kf == 0 || kf == N - 1) {
        // the box's own face: the other reading of a point within FP32 of
        // it is inside (the trilinear slope) or clamped (the direction to
        // the face, from the outside)
        ub = konst<S>(static_cast<double>(kf));
        outward = !cl[a];
        cl[a] = !cl[a];
        c[a] = std::min(kf, N - 2);
      } else if (c[a] == kf) {
        // the other cell at the nearest interior face k
        c[a] = kf - 1;
      } else if (c[a] == kf - 1) {
        c[a] = kf;
      }
    }
    f[a] = ub - static_cast<double>(c[a]);
    e[a] = cl[a] ? (u - ub) * o.h : konst<S>(0.0);
    if (outward && (k == 0.0) == (val(e[a]) > 0.0)) e[a] = -e[a];
    margin = std::min(margin, std::fabs(val(u) - k));
    if (info) info->axis_margin[a] = std::fabs(val(u) - k);
  }
  auto V = [&](int i, int j, int k) -> double {
    return static_cast<double>(o.values[(static_cast<int64_t>(c[2] + k) * N + (c[1] + j)) * N + (c[0] + i)]);
  };
  S w0[3], w1[3];
  for (int a = 0; a < 3; ++a) { w1[a] = f[a]; w0[a] = 1.0 - f[a]; }
  S val_tri = konst<S>(0.0);
  S df[3] = {konst<S>(0.0), konst<S>(0.0), konst<S>(0.0)};
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        double v = V(i, j, k);
        const S& wx = i ? w1[0] : w0[0];
        const S& wy = j ? w1[1] : w0[1];
        const S& wz = k ? w1[2] : w0[2];
        val_tri += v * (wx * wy * wz);
        df[0] += (i ? v : -v) * (wy * wz);
        df[1] += (j ? v : -v) * (wx * wz);
        df[2] += (k ? v : -v) * (wx * wy);
      }
  for (int a = 0; a < 3; ++a) n[a] = cl[a] ? konst<S>(0.0) : df[a] / o.h;
  phi = val_tri;
  S ne = norm3(e);
  if (val(ne) > 0.0) {
    phi = phi + ne;
    for (int a = 0; a < 3; ++a) n[a] = n[a] + e[a] / ne;
  }
  if (info) {
    for (int a = 0; a < 3; ++a) { info->cell[a] = c[a]; info->clamped[a] = cl[a]; }
    info->face_margin = margin;
  }
}

// Grid normal by central differences (Sec. III-A: finite differencing costs
// seven queries per sample against one): the value and cell at r, then the
// value at r +- h along each axis. A face of the grid is crossed by r + h e_a
// exactly when it is crossed by r, so the centre's face margin still flags
// every kink.
template <class S>
void sample_grid_fd(const oobject& o, const S r[3], S& phi, S n[3], SampleInfo* info) {
  S unused[3];
  sample_grid(o, r, phi, unused, info);
  for (int a = 0; a < 3; ++a) {
    S rp[3] = {r[0], r[1], r[2]}, rm[3] = {r[0], r[1], r[2]};
    rp[a] = rp[a] + o.h;
    rm[a] = rm[a] - o.h;
    S vp, vm;
    sample_grid(o, rp, vp, unused, nullptr);
    sample_grid(o, rm, vm, unused, nullptr);
    n[a] = (vp - vm) / (2.0 * o.h);
  }
}

// Mesh object (Sec. III-B): Phong signed distance rho(r) = s |r - p|. The
// closest point r* of the flat mesh is searched over every face in FP64; its
// face and region (face interior, an edge or a vertex) and the sign s of the
// flat mesh (winding number) are discrete and carry no derivative. r* is then
// formed again in the scalar type from its region's formula (projection onto
// the face plane or the edge line, or the vertex itself) with its
// barycentric weights, and the Phong point follows:
//   p = (1 - alpha) r* + alpha sum_b w_b psi_b(r*),
//   psi_b(x) = x - ((x - v_b) . n_b) n_b (the tangent plane of vertex b).
// The constraint normal is the gradient the paper states, (r - p) / rho
// (the face normal at rho = 0); the dual numbers carry the exact derivative
// of rho and of that normal through r*, the weights and the Phong point. The
// leaky rule's hand-point part takes the stated normal as the direction, as
// it takes the trilinear gradient on a grid.
struct MeshHit {
  int face = -1;
  int region = 0;  // 0 face interior, 1 edge (v0, v1), 2 vertex v0 (indices 0..2 within the face)
  int v0 = 0, v1 = 0;
  double s = 1.0;
  double dist_flat = 0.0;
  double y[3] = {0, 0, 0};  // the closest point
  // the neighbouring region of the same face nearest to the closest point
  // (interior <-> edge <-> vertex) and how far the closest point is from it
  int alt_region = 0, alt_v0 = 0, alt_v1 = 0;
  double region_margin = INFINITY;
};

// The closest point of face f to r as a hit (region from its weights).
MeshHit face_hit(const omesh& m, int f, const double r[3], double& dist) {
  MeshHit h;
  const int* t = m.faces + 3 * f;
  double w[3];
  oracle_closest_on_triangle(m.vertices + 3 * t[0], m.vertices + 3 * t[1], m.vertices + 3 * t[2], r, h.y, w);
  dist = std::sqrt((r[0] - h.y[0]) * (r[0] - h.y[0]) + (r[1] - h.y[1]) * (r[1] - h.y[1]) +
                   (r[2] - h.y[2]) * (r[2] - h.y[2]));
  h.face = f;
  int nz[3], k = 0;
  for (int j = 0; j < 3; ++j)
    if (w[j] != 0.0) nz[k++] = j;
  h.region = k == 3 ? 0 : (k == 2 ? 1 : 2);
  h.v0 = k >= 1 ? nz[0] : 0;
  h.v1 = k >= 2 ? nz[1] : 0;
  h.dist_flat = dist;
  // distance (metres) from the closest point to the nearest other region
  const double* P[3] = {m.vertices + 3 * t[0], m.vertices + 3 * t[1], m.vertices + 3 * t[2]};
  auto sub = [](const double* a, const double* b, double* o) { for (int i = 0; i < 3; ++i) o[i] = a[i] - b[i]; };
  auto dot3 = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  auto edge_param = [&](int a, int b) {  // parameter of r's projection on the line P[a] -> P[b], and |e|
    double e[3], ra[3];
    sub(P[b], P[a], e);
    sub(r, P[a], ra);
    const double ee = dot3(e, e);
    return std::make_pair(dot3(ra, e) / ee, std::sqrt(ee));
  };
  if (h.region == 0) {
    // the edge opposite the smallest weight: distance = w * height over that edge
    int j = 0;
    for (int i = 1; i < 3; ++i)
      if (w[i] < w[j]) j = i;
    const int a = (j + 1) % 3, b = (j + 2) % 3;
    double e1[3], e2[3], N[3];
    sub(P[1], P[0], e1);
    sub(P[2], P[0], e2);
    N[0] = e1[1] * e2[2] - e1[2] * e2[1];
    N[1] = e1[2] * e2[0] - e1[0] * e2[2];
    N[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double area2 = std::sqrt(dot3(N, N));
    h.alt_region = 1;
    h.alt_v0 = std::min(a, b);
    h.alt_v1 = std::max(a, b);
    h.region_margin = w[j] * area2 / edge_param(a, b).second;
  } else if (h.region == 1) {
    // the vertex at the nearer end, or the interior when r projects just inside
    const auto tp = edge_param(h.v0, h.v1);
    const double to_vertex = std::min(tp.first, 1.0 - tp.first) * tp.second;
    const int c = 3 - h.v0 - h.v1;
    double e[3], rc[3], ec[3];
    sub(P[h.v1], P[h.v0], e);
    sub(r, P[h.v0], rc);
    sub(P[c], P[h.v0], ec);
    // the in-plane direction from the edge towards the third vertex
    double perp[3];
    const double te = dot3(ec, e) / dot3(e, e);
    for (int i = 0; i < 3; ++i) perp[i] = ec[i] - te * e[i];
    const double lp = std::sqrt(dot3(perp, perp));
    const double to_interior = -dot3(rc, perp) / lp;  // > 0: r projects outside the face
    if (to_vertex <= to_interior) {
      h.alt_region = 2;
      h.alt_v0 = tp.first < 0.5 ? h.v0 : h.v1;
      h.alt_v1 = 0;
      h.region_margin = to_vertex;
    } else {
      h.alt_region = 0;
      h.region_margin = to_interior;
    }
  } else {
    // the vertex's edge whose line r projects nearest past the vertex
    double bestm = INFINITY;
    for (int o = 0; o < 3; ++o) {
      if (o == h.v0) continue;
      const auto tp = edge_param(h.v0, o);
      const double mg = -tp.first * tp.second;  // > 0: r projects before the vertex
      if (mg < bestm) {
        bestm = mg;
        h.alt_region = 1;
        h.alt_v0 = std::min(h.v0, o);
        h.alt_v1 = std::max(h.v0, o);
      }
    }
    h.region_margin = bestm;
  }
  return h;
}

// The closest point of the flat mesh (first face of least distance), and the
// nearest different point of the surface (faces that share the closest edge
// or vertex give the same point and do not count): near the medial axis the
// two are nearly equidistant and FP32 may take either.
void mesh_closest(const omesh& m, const double r[3], MeshHit& best, MeshHit& second) {
  double bd = INFINITY;
  for (int f = 0; f < m.n_faces; ++f) {
    double d;
    const MeshHit h = face_hit(m, f, r, d);
    if (d < bd) { bd = d; best = h; }
  }
  double sd = INFINITY;
  second = best;
  second.dist_flat = INFINITY;
  for (int f = 0; f < m.n_faces; ++f) {
    double d;
    const MeshHit h = face_hit(m, f, r, d);
    const double sep = std::sqrt((h.y[0] - best.y[0]) * (h.y[0] - best.y[0]) + (h.y[1] - best.y[1]) * (h.y[1] - best.y[1]) +
                                 (h.y[2] - best.y[2]) * (h.y[2] - best.y[2]));
    if (sep > 1e-9 && d < sd) { sd = d; second = h; }
  }
  best.s = second.s = oracle_winding_number(&m, r) > 0.5 ? -1.0 : 1.0;
}

template <class S> void phong_rho(const omesh& m, const MeshHit& h, const S r[3], S& rho, S n[3]) {
  const int* t = m.faces + 3 * h.face;
  const double* P[3] = {m.vertices + 3 * t[0], m.vertices + 3 * t[1], m.vertices + 3 * t[2]};
  const double* Nv[3] = {m.normals + 3 * t[0], m.normals + 3 * t[1], m.normals + 3 * t[2]};
  double e1[3], e2[3], N[3];
  for (int i = 0; i < 3; ++i) { e1[i] = P[1][i] - P[0][i]; e2[i] = P[2][i] - P[0][i]; }
  N[0] = e1[1] * e2[2] - e1[2] * e2[1];
  N[1] = e1[2] * e2[0] - e1[0] * e2[2];
  N[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
  S x[3], w[3] = {konst<S>(0.0), konst<S>(0.0), konst<S>(0.0)};
  if (h.region == 0) {
    // projection onto the face plane, weights from the sub-triangle areas
    S off = konst<S>(0.0);
    for (int i = 0; i < 3; ++i) off += (r[i] - P[0][i]) * N[i];
    for (int i = 0; i < 3; ++i) x[i] = r[i] - (off / nn) * N[i];
    for (int j = 0; j < 2; ++j) {
      // w_j = ((P[j+2] - P[j+1]) x (x - P[j+1])) . N / |N|^2
      const double* A = P[(j + 1) % 3];
      const double* Bv = P[(j + 2) % 3];
      const double u[3] = {Bv[0] - A[0], Bv[1] - A[1], Bv[2] - A[2]};
      const S v[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
      const S c0 = u[1] * v[2] - u[2] * v[1], c1 = u[2] * v[0] - u[0] * v[2], c2 = u[0] * v[1] - u[1] * v[0];
      w[j] = (c0 * N[0] + c1 * N[1] + c2 * N[2]) / nn;
    }
    w[2] = 1.0 - w[0] - w[1];
  } else if (h.region == 1) {
    // projection onto the edge's line
    const double* A = P[h.v0];
    const double* Bv = P[h.v1];
    const double d[3] = {Bv[0] - A[0], Bv[1] - A[1], Bv[2] - A[2]};
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    S tp = konst<S>(0.0);
    for (int i = 0; i < 3; ++i) tp += (r[i] - A[i]) * d[i];
    tp = tp / dd;
    for (int i = 0; i < 3; ++i) x[i] = A[i] + tp * d[i];
    w[h.v0] = 1.0 - tp;
    w[h.v1] = tp;
  } else {
    for (int i = 0; i < 3; ++i) x[i] = konst<S>(P[h.v0][i]);
    w[h.v0] = konst<S>(1.0);
  }
  // Phong point
  S curved[3] = {konst<S>(0.0), konst<S>(0.0), konst<S>(0.0)};
  for (int b = 0; b < 3; ++b) {
    S hb = konst<S>(0.0);
    for (int i = 0; i < 3; ++i) hb += (x[i] - P[b][i]) * Nv[b][i];
    for (int i = 0; i < 3; ++i) curved[i] += w[b] * (x[i] - hb * Nv[b][i]);
  }
  S dv[3];
  for (int i = 0; i < 3; ++i) dv[i] = r[i] - ((1.0 - m.alpha) * x[i] + m.alpha * curved[i]);
  const S d2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
  if (val(d2) > 0.0) {
    const S dist = sqrt_(d2);
    rho = h.s * dist;
    for (int i = 0; i < 3; ++i) n[i] = dv[i] / rho;
  } else {
    rho = konst<S>(0.0);
    const double l = std::sqrt(nn);
    for (int i = 0; i < 3; ++i) n[i] = konst<S>(N[i] / l);
  }
}

template <class S>
void sample_mesh(const oobject& o, const S r[3], S& phi, S n[3], SampleInfo* info) {
  const double rv[3] = {val(r[0]), val(r[1]), val(r[2])};
  MeshHit best, second;
  mesh_closest(*o.mesh, rv, best, second);
  const double gap = second.dist_flat - best.dist_flat;
  MeshHit h = (info && info->flip_alt && std::isfinite(gap)) ? second : best;
  if (info && info->flip_sign) h.s = -h.s;
  if (info && info->flip_region) {
    h.region = best.alt_region;
    h.v0 = best.alt_v0;
    h.v1 = best.alt_v1;
  }
  phong_rho(*o.mesh, h, r, phi, n);
  if (info) {
    info->sign_margin = best.dist_flat;
    info->alt_margin = std::isfinite(gap) ? gap : 1e30;
    info->region_margin = std::fabs(best.region_margin);
    // the discrete state, for the signature: the closest feature (a face, an
    // edge by its sorted vertices, a vertex; faces that share the feature
    // give the same point) and the sign
    const int* t = o.mesh->faces + 3 * h.face;
    const int a = t[h.v0], b = t[h.v1];
    info->cell[0] = h.region == 0 ? h.face : std::min(a, b);
    info->cell[1] = h.region == 1 ? std::max(a, b) : 0;
    info->cell[2] = h.region;
    info->clamped[0] = h.s > 0.0 ? 1 : 0;
  }
}

template <class S>
void sample_object(const oobject& o, const S r[3], S& phi, S n[3], SampleInfo* info) {
  switch (o.kind) {
    case OBJ_MESH:
      sample_mesh(o, r, phi, n, info);
      return;
    case OBJ_GRID:
      if (o.fd_normal) sample_grid_fd(o, r, phi, n, info);
      else sample_grid(o, r, phi, n, info);
      return;
    case OBJ_SPHERE: {
      S a[3];
      for (int i = 0; i < 3; ++i) a[i] = r[i] - o.center[i];
      S l = norm3(a);
      phi = l - o.radius;
      for (int i = 0; i < 3; ++i) n[i] = (val(l) > 0.0) ? a[i] / l : konst<S>(0.0);
      return;
    }
    case OBJ_PLANE: {
      phi = r[0] * o.normal[0] + r[1] * o.normal[1] + r[2] * o.normal[2] - o.offset;
      for (int i = 0; i < 3; ++i) n[i] = konst<S>(o.normal[i]);
      return;
    }
    case OBJ_BOX: {
      // exact box SDF: outside |max(q, 0)|, inside max_i q_i, q = |y| - half
      S y[3], qv[3];
      double sg[3];
      for (int i = 0; i < 3; ++i) {
        y[i] = r[i] - o.center[i];
        sg[i] = val(y[i]) >= 0.0 ? 1.0 : -1.0;
        qv[i] = sg[i] * y[i] - o.half[i];
      }
      S pos[3];
      bool any_out = false;
      for (int i = 0; i < 3; ++i) {
        pos[i] = val(qv[i]) > 0.0 ? qv[i] : konst<S>(0.0);
        any_out = any_out || val(qv[i]) > 0.0;
      }
      if (any_out) {
        S l = norm3(pos);
        phi = l;
        for (int i = 0; i < 3; ++i) n[i] = sg[i] * (pos[i] / l);
      } else {
        int m = 0;
        for (int i = 1; i < 3; ++i) if (val(qv[i]) > val(qv[m])) m = i;
        phi = qv[m];
        for (int i = 0; i < 3; ++i) n[i] = konst<S>(i == m ? sg[i] : 0.0);
      }
      return;
    }
    default:
      phi = konst<S>(0.0);
      for (int i = 0; i < 3; ++i) n[i] = konst<S>(0.0);
  }
}

double inertia_over_mass(const oobject& o) {
  if (o.inertia_over_mass > 0.0 || o.kind != OBJ_GRID) return o.inertia_over_mass;
  // isotropic inertia of a uniform ball of the object's volume:
  // I/m = 2/5 R_eq^2, V = h^3 * (number of vertices with phi < 0)
  const int64_t n3 = static_cast<int64_t>(o.n) * o.n * o.n;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n3; ++i) cnt += (o.values[i] < 0.0f) ? 1 : 0;
  const double V = o.h * o.h * o.h * static_cast<double>(cnt);
  const double Req = std::cbrt(3.0 * V / (4.0 * M_PI));
  return 0.4 * Req * Req;
}

// ---------------------------------------------------------------------------
// object orientation: rotation vector theta, R = I + A [t]x + B [t]x^2 with
// A = sin|t|/|t| and B = (1 - cos|t|)/|t|^2; power series below |t| = 0.5
// ---------------------------------------------------------------------------
template <class S> void rotation_matrix(const S th[3], S R[9]) {
  S s = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  S A, B;
  if (val(s) < 0.25) {
    S s2 = s * s, s3 = s2 * s, s4 = s3 * s;
    A = 1.0 - s / 6.0 + s2 / 120.0 - s3 / 5040.0 + s4 / 362880.0;
    B = 0.5 - s / 24.0 + s2 / 720.0 - s3 / 40320.0 + s4 / 3628800.0;
  } else {
    S t = sqrt_(s);
    A = sin_(t) / t;
    B = (1.0 - cos_(t)) / s;
  }
  S K[9] = {konst<S>(0.0), -th[2], th[1], th[2], konst<S>(0.0), -th[0], -th[1], th[0], konst<S>(0.0)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S k2 = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
      R[3 * i + j] = ((i == j) ? 1.0 : 0.0) + A * K[3 * i + j] + B * k2;
    }
}

// ---------------------------------------------------------------------------
// one grasp step for one candidate
// ---------------------------------------------------------------------------
struct Trace {
  double* poses = nullptr;    // [M][K+1][6]
  double* samples = nullptr;  // [M][K][Nc][6]
  double* p_world = nullptr;  // [Nc][3]
  double min_abs_d = 1e30;      // min |d + eps| over samples with w > w_min: distance from the activation
  double min_face = 1e30;      // penetrating samples: their gradient sets a correction
  double min_face_all = 1e30;  // every sample with w > w_min: the leak reaches its gradient
  uint64_t signature = 1469598103934665603ull;  // FNV-1a over discrete decisions
  // readings of ambiguous samples to take (flips of this candidate) and the
  // report of the samples that are ambiguous at FP32 resolution
  const oflip* flips = nullptr;
  int n_flips = 0;
  double kink_d = -1.0, kink_face = -1.0;
  std::vector<oamb>* amb = nullptr;
  // flips of sample (m, k, i): bit 0 = the other side of the activation
  // d = -eps, bit 1 + a = the other cell along axis a, bit 4 the other side
  // of the friction cone, bit 5 of the friction floor, bit 6 of a mesh's
  // flat surface, bit 7 the nearest different point of a mesh, bit 8 the
  // neighbouring region of a mesh's closest point
  int flips_of(int m, int k, int i) const {
    int f = 0;
    for (int j = 0; j < n_flips; ++j)
      if (flips[j].m == m && flips[j].k == k && flips[j].i == i) f |= 1 << flips[j].what;
    return f;
  }
  void report_friction(int m, int k, int i, double gap) {
    if (amb && std::fabs(gap) < kink_d) amb->push_back(oamb{m, k, i, 4, std::fabs(gap), 1});
  }
  void report_slide(int m, int k, int i, double gap) {
    if (amb && std::fabs(gap) < kink_d) amb->push_back(oamb{m, k, i, 5, std::fabs(gap), 1});
  }
  // gap: d + eps, the distance from the activation
  void report(int m, int k, int i, double gap, const SampleInfo& info, bool pen) {
    if (!amb) return;
    if (std::fabs(gap) < kink_d) amb->push_back(oamb{m, k, i, 0, std::fabs(gap), pen ? 1 : 0});
    for (int a = 0; a < 3; ++a)
      if (info.axis_margin[a] < kink_face) amb->push_back(oamb{m, k, i, 1 + a, info.axis_margin[a], pen ? 1 : 0});
    if (info.sign_margin < kink_d) amb->push_back(oamb{m, k, i, 6, info.sign_margin, pen ? 1 : 0});
    if (info.alt_margin < kink_d) amb->push_back(oamb{m, k, i, 7, info.alt_margin, pen ? 1 : 0});
    if (info.region_margin < kink_d) amb->push_back(oamb{m, k, i, 8, info.region_margin, pen ? 1 : 0});
  }
  void mix(uint64_t x) {
    for (int i = 0; i < 8; ++i) { signature ^= (x >> (8 * i)) & 0xff; signature *= 1099511628211ull; }
  }
};

// The part of d's tangent that comes from the hand point p alone:
// dd/dp = (R grad(phi))^T = g^T, so d_hand = g . dp (value d).
inline double hand_part(const double& d, const double*, const double*) { return d; }
template <int N> Dual<N> hand_part(const Dual<N>& d, const Dual<N>* g, const Dual<N>* p) {
  Dual<N> r(d.v);
  for (int t = 0; t < N; ++t) r.d[t] = g[0].v * p[0].d[t] + g[1].v * p[1].d[t] + g[2].v * p[2].d[t];
  return r;
}


// C = max(0, -d) with the leaky derivative rule (Sec. III-C, "Leaky
// gradient"), for a constraint that counts as penetrating (pen): value -d and
// tangent -dd; otherwise value 0 and tangent -alpha times the hand-point part
// of dd. The leak is a surrogate derivative for hand points that do not
// touch the object; along the object's pose from one projection iteration to
// the next the derivative stays exact (with one iteration the pose carries no
// tangent and the two coincide).
// pen: d < -eps with eps the contact tolerance (see contact_tol), unless a
// flip takes the other reading of a sample within rounding of -eps. The
// tolerance keeps a constraint that a projection has just resolved (d = 0 up
// to rounding) out of the active set: at d = 0 the active state, and with it
// the derivative rule and the averaging count, would be decided by rounding.
template <class S> S leaky_penetration(const S& d, const S& d_hand, double alpha, bool pen) {
  S c = pen ? -d : -alpha * d_hand;
  if (!pen) c.v = 0.0;
  return c;
}
template <> double leaky_penetration<double>(const double& d, const double&, double, bool pen) {
  return pen ? -d : 0.0;
}

// The contact tolerance: a sample penetrates (counts as an active
// constraint) when d < -contact_tol(P) = -5e-3 dt v0, half a percent of a
// test's displacement.
inline double contact_tol(const oparams& P) { return kContactTol * P.dt * P.v0; }

// Coulomb friction of one active contact (Sec. III-C cites a friction model
// without stating it; read here as positional friction in position-based
// dynamics). The object's material point at the contact, at r in the object
// frame, started the step at r (rest pose) and is now at the hand point p:
// it moved by dp = p - r. Its tangential part dp_t = dp - (dp . n) n, with
// n = g / |g| the contact normal, is removed up to the Coulomb bound mu C:
// wholly while |dp_t| <= mu C (static friction), by mu C along it otherwise
// (kinetic), as the Eq. (1) correction of a positional constraint along
// t = dp_t / |dp_t|: lambda_t = -min(|dp_t|, mu C) / w_t with
// w_t = |t|^2 + |a x t|^2 / (I/m). Adds (lambda_t t, lambda_t a x t) to the
// sums of corrections. A slide no longer than smin (a thousandth of the
// test displacement dt v0) has no direction: the contact gets no friction.
// Without that floor a slide that is zero in exact arithmetic (a test
// moving along a flat face's normal) would take its direction from rounding.
template <class S>
void add_friction(const S p[3], const S r[3], const S a[3], const S g[3], const S& C, double mu, double Im,
                  double smin, S Wl[3], S Wa[3], Trace* tr = nullptr, int m = 0, int k = 0, int i = 0) {
  const S gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  if (!(val(gg) > 0.0)) return;
  const S ng = sqrt_(gg);
  S nh[3], dp[3], dpt[3];
  for (int j = 0; j < 3; ++j) { nh[j] = g[j] / ng; dp[j] = p[j] - r[j]; }
  const S sn = dp[0] * nh[0] + dp[1] * nh[1] + dp[2] * nh[2];
  for (int j = 0; j < 3; ++j) dpt[j] = dp[j] - sn * nh[j];
  const S tl2 = dpt[0] * dpt[0] + dpt[1] * dpt[1] + dpt[2] * dpt[2];
  if (!(val(tl2) > 0.0)) return;
  const S tl = sqrt_(tl2);
  // the floor: a flip takes the other side of it within rounding
  bool slides = val(tl) > smin;
  if (tr) {
    if (tr->flips_of(m, k, i) & (1 << 5)) slides = !slides;
    tr->report_slide(m, k, i, val(tl) - smin);
  }
  if (!slides) return;
  S th[3];
  for (int j = 0; j < 3; ++j) th[j] = dpt[j] / tl;
  S ut[3];
  ut[0] = a[1] * th[2] - a[2] * th[1];
  ut[1] = a[2] * th[0] - a[0] * th[2];
  ut[2] = a[0] * th[1] - a[1] * th[0];
  const S wt = (th[0] * th[0] + th[1] * th[1] + th[2] * th[2]) + (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]) / Im;
  // static while the displacement is within the cone, kinetic beyond it
  // (a flip takes the other side of a switch within rounding)
  bool stat = val(tl) <= mu * val(C);
  if (tr) {
    if (tr->flips_of(m, k, i) & (1 << 4)) stat = !stat;
    tr->report_friction(m, k, i, val(tl) - mu * val(C));
  }
  const S delta = stat ? tl : mu * C;
  const S lt = -delta / wt;
  for (int j = 0; j < 3; ++j) { Wl[j] += lt * th[j]; Wa[j] += lt * ut[j]; }
}

template <class S>
void candidate_step(const ohand& h, const oobject& o, double Im, const oparams& P, const S* q,
                    S& loss, S terms[4], Trace* tr) {
  const int Nc = h.n_contacts;
  const int nd = 6 + h.n_links - 1;
  // 1. forward kinematics: hand points p_i (the hand is static during the step)
  std::vector<Xf<S>> T;
  forward_kinematics(h, q, T);
  std::vector<S> p(3 * static_cast<size_t>(Nc));
  for (int i = 0; i < Nc; ++i) apply_xf(T[h.contact_link[i]], h.contact_local + 3 * i, &p[3 * i]);
  if (tr && tr->p_world)
    for (int i = 0; i < 3 * Nc; ++i) tr->p_world[i] = val(p[i]);

  // 2. penetration of the hand at the object's rest pose, with dilation:
  //    C0_i = max(0, -(phi(p_i) - r)); L_pen = 1/2 sum C0_i^2
  //    (the same samples as the rest test's first iteration, m = 6, k = 0,
  //    so a flip of one of those applies here too)
  S Lpen = konst<S>(0.0);
  for (int i = 0; i < Nc; ++i) {
    S phi, n[3];
    SampleInfo info;
    const int fl = tr ? tr->flips_of(kSims - 1, 0, i) : 0;
    info.flip_axes = fl >> 1;
    info.flip_sign = (fl >> 6) & 1;
    info.flip_alt = (fl >> 7) & 1;
    info.flip_region = (fl >> 8) & 1;
    sample_object(o, &p[3 * i], phi, n, &info);
    S d = phi - P.r_dil;
    // 1/2 C0^2 is smooth at d = 0: no reading of the side is needed here
    if (val(d) < 0.0) Lpen += 0.5 * (d * d);
  }
  const double eps = contact_tol(P);

  // 3. M velocity-test simulations (Sec. IV-A), each one PBD step (Sec. III-C)
  const double dirs[kSims][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {0, 0, 1}, {0, 0, -1}, {0, 0, 0}};
  // Gauss-Seidel order: contacts stable-sorted by link
  std::vector<int> order(Nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h.contact_link[a] < h.contact_link[b]; });
  S Lstable = konst<S>(0.0);
  for (int m = 0; m < kSims; ++m) {
    // symplectic-Euler prediction from the canonical pose with velocity v0_m
    S x[3], th[3];
    for (int a = 0; a < 3; ++a) { x[a] = konst<S>(P.dt * P.v0 * dirs[m][a]); th[a] = konst<S>(0.0); }
    for (int k = 0; k < P.K; ++k) {
      if (tr && tr->poses)
        for (int a = 0; a < 3; ++a) {
          tr->poses[(m * (P.K + 1) + k) * 6 + a] = val(x[a]);
          tr->poses[(m * (P.K + 1) + k) * 6 + 3 + a] = val(th[a]);
        }
      if (P.projection == 1) {
        // Gauss-Seidel: each constraint's Eq. (1) update applied at once, so
        // the next constraint sees the pose the previous ones left
        for (int oi = 0; oi < Nc; ++oi) {
          const int i = order[oi];
          S R[9];
          rotation_matrix(th, R);
          S a[3], r[3];
          for (int j = 0; j < 3; ++j) a[j] = p[3 * i + j] - x[j];
          for (int j = 0; j < 3; ++j) r[j] = R[j] * a[0] + R[3 + j] * a[1] + R[6 + j] * a[2];
          S phi, nrm[3];
          SampleInfo info;
          const int fl = tr ? tr->flips_of(m, k, i) : 0;
          info.flip_axes = fl >> 1;
          info.flip_sign = (fl >> 6) & 1;
          info.flip_alt = (fl >> 7) & 1;
          info.flip_region = (fl >> 8) & 1;
          sample_object(o, r, phi, nrm, &info);
          S d = phi - P.r_dil;
          const bool pen = (val(d) < -eps) != ((fl & 1) != 0);
          S g[3], u[3];
          for (int j = 0; j < 3; ++j) g[j] = R[3 * j] * nrm[0] + R[3 * j + 1] * nrm[1] + R[3 * j + 2] * nrm[2];
          S C = leaky_penetration(d, hand_part(d, g, &p[3 * i]), P.alpha_leak, pen);
          u[0] = a[1] * g[2] - a[2] * g[1];
          u[1] = a[2] * g[0] - a[0] * g[2];
          u[2] = a[0] * g[1] - a[1] * g[0];
          S w = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / Im;
          S lam = konst<S>(0.0);
          const bool active = val(w) > P.w_min;
          if (active) {
            lam = -C / w;
            S Wl[3] = {lam * g[0], lam * g[1], lam * g[2]};
            S Wa[3] = {lam * u[0], lam * u[1], lam * u[2]};
            // friction from the same sample, added to this constraint's update
            if (P.mu > 0.0) add_friction(&p[3 * i], r, a, g, C, P.mu, Im, kSlideMin * P.dt * P.v0, Wl, Wa, tr, m, k, i);
            for (int j = 0; j < 3; ++j) {
              x[j] = x[j] + P.omega * Wl[j];
              th[j] = th[j] + (P.omega / Im) * Wa[j];
            }
          }
          if (tr) {
            if (tr->samples) {
              double* s = tr->samples + ((static_cast<size_t>(m) * P.K + k) * Nc + i) * 6;
              s[0] = val(d); s[1] = val(g[0]); s[2] = val(g[1]); s[3] = val(g[2]);
              s[4] = val(w); s[5] = val(lam);
            }
            if (active) tr->min_abs_d = std::min(tr->min_abs_d, std::fabs(val(d) + eps));
            if (active && val(d) < -eps) tr->min_face = std::min(tr->min_face, info.face_margin);
            if (active) tr->min_face_all = std::min(tr->min_face_all, info.face_margin);
            if (active) tr->report(m, k, i, val(d) + eps, info, pen);
            tr->mix(static_cast<uint64_t>(info.cell[0]) | (static_cast<uint64_t>(info.cell[1]) << 16) |
                    (static_cast<uint64_t>(info.cell[2]) << 32) |
                    (static_cast<uint64_t>(info.clamped[0] + 2 * info.clamped[1] + 4 * info.clamped[2]) << 48) |
                    (static_cast<uint64_t>(val(d) < -eps) << 52) | (static_cast<uint64_t>(active) << 53));
          }
        }
        continue;
      }
      S R[9];
      rotation_matrix(th, R);
      S Wl[3] = {konst<S>(0.0), konst<S>(0.0), konst<S>(0.0)};
      S Wa[3] = {konst<S>(0.0), konst<S>(0.0), konst<S>(0.0)};
      int n_active = 0;
      for (int i = 0; i < Nc; ++i) {
        // hand point in the object frame: r_i = R(theta)^-1 (p_i - x)
        S a[3], r[3];
        for (int j = 0; j < 3; ++j) a[j] = p[3 * i + j] - x[j];
        for (int j = 0; j < 3; ++j) r[j] = R[j] * a[0] + R[3 + j] * a[1] + R[6 + j] * a[2];
        S phi, nrm[3];
        SampleInfo info;
        const int fl = tr ? tr->flips_of(m, k, i) : 0;
        info.flip_axes = fl >> 1;
        info.flip_sign = (fl >> 6) & 1;
        info.flip_alt = (fl >> 7) & 1;
        info.flip_region = (fl >> 8) & 1;
        sample_object(o, r, phi, nrm, &info);
        // dilated surface: the r_dil level set (Sec. III-B, "SDF dilation")
        S d = phi - P.r_dil;
        const bool pen = (val(d) < -eps) != ((fl & 1) != 0);
        // constraint Jacobian J_C = (dC/dx, dC/dtheta) = (g, a x g), g = R grad(phi)
        S g[3], u[3];
        for (int j = 0; j < 3; ++j) g[j] = R[3 * j] * nrm[0] + R[3 * j + 1] * nrm[1] + R[3 * j + 2] * nrm[2];
        S C = leaky_penetration(d, hand_part(d, g, &p[3 * i]), P.alpha_leak, pen);
        u[0] = a[1] * g[2] - a[2] * g[1];
        u[1] = a[2] * g[0] - a[0] * g[2];
        u[2] = a[0] * g[1] - a[1] * g[0];
        // Eq. (1) with M = diag(1, 1, 1, I/m, I/m, I/m):
        // [dx; dtheta] = -M^-1 J^T (J M^-1 J^T)^-1 C = lambda (g, u / (I/m)), lambda = -C / w
        S w = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / Im;
        S lam = konst<S>(0.0);
        const bool active = val(w) > P.w_min;
        if (active) {
          lam = -C / w;
          for (int j = 0; j < 3; ++j) { Wl[j] += lam * g[j]; Wa[j] += lam * u[j]; }
          if (pen) ++n_active;
          if (P.mu > 0.0) add_friction(&p[3 * i], r, a, g, C, P.mu, Im, kSlideMin * P.dt * P.v0, Wl, Wa, tr, m, k, i);
        }
        if (tr) {
          if (tr->samples) {
            double* s = tr->samples + ((static_cast<size_t>(m) * P.K + k) * Nc + i) * 6;
            s[0] = val(d); s[1] = val(g[0]); s[2] = val(g[1]); s[3] = val(g[2]);
            s[4] = val(w); s[5] = val(lam);
          }
          if (active) tr->min_abs_d = std::min(tr->min_abs_d, std::fabs(val(d) + eps));
          if (active && val(d) < -eps) tr->min_face = std::min(tr->min_face, info.face_margin);
          if (active) tr->min_face_all = std::min(tr->min_face_all, info.face_margin);
          if (active) tr->report(m, k, i, val(d) + eps, info, pen);
          tr->mix(static_cast<uint64_t>(info.cell[0]) | (static_cast<uint64_t>(info.cell[1]) << 16) |
                  (static_cast<uint64_t>(info.cell[2]) << 32) |
                  (static_cast<uint64_t>(info.clamped[0] + 2 * info.clamped[1] + 4 * info.clamped[2]) << 48) |
                  (static_cast<uint64_t>(val(d) < -eps) << 52) | (static_cast<uint64_t>(active) << 53));
        }
      }
      // all corrections at the same pose, averaged over the active constraints,
      // relaxed by omega
      const double avg = P.omega / static_cast<double>(std::max(n_active, 1));
      for (int j = 0; j < 3; ++j) {
        x[j] = x[j] + avg * Wl[j];
        th[j] = th[j] + (avg / Im) * Wa[j];
      }
    }
    if (tr && tr->poses)
      for (int a = 0; a < 3; ++a) {
        tr->poses[(m * (P.K + 1) + P.K) * 6 + a] = val(x[a]);
        tr->poses[(m * (P.K + 1) + P.K) * 6 + 3 + a] = val(th[a]);
      }
    // velocities from positions: x' = (x+ - x-)/dt with x- = 0 (Sec. III-C)
    S v[3], wv[3];
    for (int a = 0; a < 3; ++a) { v[a] = x[a] / P.dt; wv[a] = th[a] / P.dt; }
    // L_stable = sum_m (|x'_m| + |theta'_m|) / M (Sec. IV-A)
    Lstable += (norm3(v) + norm3(wv)) / static_cast<double>(kSims);
  }

  // 4. joint losses over finger joints (Sec. IV-A)
  S rs = konst<S>(0.0);
  S Llimit = konst<S>(0.0);
  for (int j = 6; j < nd; ++j) {
    S dm = q[j] - 0.5 * (h.q_up[j] + h.q_low[j]);
    rs += dm * dm;
    if (val(q[j]) > h.q_up[j]) Llimit += q[j] - h.q_up[j];
    if (val(q[j]) < h.q_low[j]) Llimit += h.q_low[j] - q[j];
    if (tr) tr->mix(static_cast<uint64_t>(j) << 8 | (val(q[j]) > h.q_up[j]) | (val(q[j]) < h.q_low[j]) << 1);
  }
  S Lrange = (val(rs) > 0.0) ? sqrt_(rs) : konst<S>(0.0);

  terms[0] = Lstable;
  terms[1] = Lpen;
  terms[2] = Lrange;
  terms[3] = Llimit;
  loss = P.w_stable * Lstable + P.w_pen * Lpen + P.w_range * Lrange + P.w_limit * Llimit;
}

bool valid_hand(const ohand* h) {
  if (!h || h->n_links < 1 || h->n_contacts < 0 || !h->parent || !h->joint_origin || !h->joint_axis ||
      !h->q_low || !h->q_up || (h->n_contacts > 0 && (!h->contact_local || !h->contact_link)))
    return false;
  if (h->parent[0] != -1) return false;
  for (int l = 1; l < h->n_links; ++l)
    if (h->parent[l] < 0 || h->parent[l] >= l) return false;
  for (int i = 0; i < h->n_contacts; ++i)
    if (h->contact_link[i] < 0 || h->contact_link[i] >= h->n_links) return false;
  return true;
}

bool valid_obj(const oobject* o) {
  if (!o) return false;
  if (o->kind == OBJ_GRID) return o->n >= 2 && o->h > 0.0 && o->values && (o->fd_normal == 0 || o->fd_normal == 1);
  if (o->kind == OBJ_MESH)
    return o->mesh && o->mesh->n_faces >= 1 && o->mesh->vertices && o->mesh->normals && o->mesh->faces &&
           o->inertia_over_mass > 0.0;
  return o->kind >= OBJ_SPHERE && o->kind <= OBJ_BOX;
}

template <int N>
void step_dual(const ohand& h, const oobject& o, double Im, const oparams& P, const double* q,
               double* loss, double* terms, double* grad, double* margins, Trace* ext = nullptr) {
  const int nd = 6 + h.n_links - 1;
  std::vector<Dual<N>> qd(nd);
  for (int j = 0; j < nd; ++j) { qd[j] = Dual<N>(q[j]); qd[j].d[j] = 1.0; }
  Dual<N> L, t4[4];
  Trace own;
  Trace& tr = ext ? *ext : own;
  candidate_step(h, o, Im, P, qd.data(), L, t4, (margins || ext) ? &tr : nullptr);
  *loss = L.v;
  if (terms) for (int i = 0; i < 4; ++i) terms[i] = t4[i].v;
  for (int j = 0; j < nd; ++j) grad[j] = L.d[j];
  if (margins) { margins[0] = tr.min_abs_d; margins[1] = tr.min_face; margins[2] = tr.min_face_all; }
}

void step_one(const ohand& h, const oobject& o, double Im, const oparams& P, const double* q,
              double* loss, double* terms, double* grad, double* margins, Trace* ext = nullptr) {
  const int nd = 6 + h.n_links - 1;
  if (!grad) {
    double L, t4[4];
    Trace own;
    Trace& tr = ext ? *ext : own;
    candidate_step(h, o, Im, P, q, L, t4, (margins || ext) ? &tr : nullptr);
    *loss = L;
    if (terms) for (int i = 0; i < 4; ++i) terms[i] = t4[i];
    if (margins) { margins[0] = tr.min_abs_d; margins[1] = tr.min_face; margins[2] = tr.min_face_all; }
    return;
  }
  if (nd <= 8) step_dual<8>(h, o, Im, P, q, loss, terms, grad, margins, ext);
  else if (nd <= 16) step_dual<16>(h, o, Im, P, q, loss, terms, grad, margins, ext);
  else if (nd <= 24) step_dual<24>(h, o, Im, P, q, loss, terms, grad, margins, ext);
  else if (nd <= 32) step_dual<32>(h, o, Im, P, q, loss, terms, grad, margins, ext);
  else step_dual<40>(h, o, Im, P, q, loss, terms, grad, margins, ext);
}

int set_threads(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // namespace

extern "C" {

int oracle_fk(const ohand* hand, int B, const double* q, double* p_out, double* frames_out) {
  if (!valid_hand(hand) || B < 0 || (B > 0 && (!q || !p_out))) return -1;
  const int nd = 6 + hand->n_links - 1, L = hand->n_links, Nc = hand->n_contacts;
  for (int b = 0; b < B; ++b) {
    std::vector<Xf<double>> T;
    forward_kinematics(*hand, q + static_cast<size_t>(b) * nd, T);
    for (int i = 0; i < Nc; ++i)
      apply_xf(T[hand->contact_link[i]], hand->contact_local + 3 * i, p_out + (static_cast<size_t>(b) * Nc + i) * 3);
    if (frames_out)
      for (int l = 0; l < L; ++l)
        for (int i = 0; i < 3; ++i) {
          for (int j = 0; j < 3; ++j) frames_out[(static_cast<size_t>(b) * L + l) * 12 + 4 * i + j] = T[l].R[3 * i + j];
          frames_out[(static_cast<size_t>(b) * L + l) * 12 + 4 * i + 3] = T[l].t[i];
        }
  }
  return 0;
}

int oracle_sample(const oobject* obj, int n, const double* r, double* phi, double* grad, double* hess,
                  double* face_margin) {
  if (!valid_obj(obj) || n < 0 || (n > 0 && (!r || !phi || !grad))) return -1;
  for (int i = 0; i < n; ++i) {
    SampleInfo info;
    if (hess) {
      Dual<3> rd[3], ph, nr[3];
      for (int a = 0; a < 3; ++a) { rd[a] = Dual<3>(r[3 * i + a]); rd[a].d[a] = 1.0; }
      sample_object(*obj, rd, ph, nr, &info);
      phi[i] = ph.v;
      for (int a = 0; a < 3; ++a) {
        grad[3 * i + a] = nr[a].v;
        for (int b = 0; b < 3; ++b) hess[9 * i + 3 * a + b] = nr[a].d[b];
      }
    } else {
      double n3[3];
      sample_object(*obj, r + 3 * i, phi[i], n3, &info);
      for (int a = 0; a < 3; ++a) grad[3 * i + a] = n3[a];
    }
    if (face_margin) face_margin[i] = info.face_margin;
  }
  return 0;
}

double oracle_inertia_over_mass(const oobject* obj) {
  if (!valid_obj(obj)) return -1.0;
  return inertia_over_mass(*obj);
}

int oracle_step(const ohand* hand, const oobject* obj, const oparams* prm, int B, const double* q,
                double* loss, double* terms, double* grad, double* margins, int n_threads) {
  if (!valid_hand(hand) || !valid_obj(obj) || !prm || B < 0 || (B > 0 && (!q || !loss)) || prm->K < 1)
    return -1;
  const double Im = inertia_over_mass(*obj);
  if (!(Im > 0.0)) return -2;
  const int nd = 6 + hand->n_links - 1;
  const int nt = set_threads(n_threads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int b = 0; b < B; ++b)
    step_one(*hand, *obj, Im, *prm, q + static_cast<size_t>(b) * nd, loss + b, terms ? terms + 4 * b : nullptr,
             grad ? grad + static_cast<size_t>(b) * nd : nullptr, margins ? margins + 3 * b : nullptr);
  return 0;
}

int oracle_step_ex(const ohand* hand, const oobject* obj, const oparams* prm, int B, const double* q,
                   double* loss, double* terms, double* grad, int n_flips, const int* flip_b, const oflip* flips,
                   double kink_d, double kink_face, int max_amb, oamb* amb, int* n_amb, int n_threads) {
  if (!valid_hand(hand) || !valid_obj(obj) || !prm || B < 0 || (B > 0 && (!q || !loss)) || prm->K < 1 ||
      n_flips < 0 || (n_flips > 0 && (!flip_b || !flips)) || max_amb < 0 || (max_amb > 0 && amb && !n_amb))
    return -1;
  for (int j = 0; j < n_flips; ++j)
    if (flip_b[j] < 0 || flip_b[j] >= B || flips[j].what < 0 || flips[j].what > 8) return -1;
  const double Im = inertia_over_mass(*obj);
  if (!(Im > 0.0)) return -2;
  const int nd = 6 + hand->n_links - 1;
  // the flips of each candidate, in input order
  std::vector<std::vector<oflip>> per(B);
  for (int j = 0; j < n_flips; ++j) per[flip_b[j]].push_back(flips[j]);
  const int nt = set_threads(n_threads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int b = 0; b < B; ++b) {
    std::vector<oamb> found;
    Trace tr;
    tr.flips = per[b].data();
    tr.n_flips = static_cast<int>(per[b].size());
    tr.kink_d = kink_d;
    tr.kink_face = kink_face;
    tr.amb = &found;
    step_one(*hand, *obj, Im, *prm, q + static_cast<size_t>(b) * nd, loss + b, terms ? terms + 4 * b : nullptr,
             grad ? grad + static_cast<size_t>(b) * nd : nullptr, nullptr, &tr);
    if (n_amb) n_amb[b] = static_cast<int>(found.size());
    if (amb)
      for (int j = 0; j < std::min<int>(max_amb, static_cast<int>(found.size())); ++j)
        amb[static_cast<size_t>(b) * max_amb + j] = found[j];
  }
  return 0;
}

int oracle_trace(const ohand* hand, const oobject* obj, const oparams* prm, const double* q, double* poses,
                 double* samples, double* p_world) {
  if (!valid_hand(hand) || !valid_obj(obj) || !prm || !q || prm->K < 1) return -1;
  const double Im = inertia_over_mass(*obj);
  if (!(Im > 0.0)) return -2;
  Trace tr;
  tr.poses = poses;
  tr.samples = samples;
  tr.p_world = p_world;
  double L, t4[4];
  candidate_step(*hand, *obj, Im, *prm, q, L, t4, &tr);
  return 0;
}

int oracle_fd_grad(const ohand* hand, const oobject* obj, const oparams* prm, int B, const double* q,
                   double fd_h, double* grad, int* excluded, int n_threads) {
  if (!valid_hand(hand) || !valid_obj(obj) || !prm || B < 0 || (B > 0 && (!q || !grad)) || !(fd_h > 0.0))
    return -1;
  const double Im = inertia_over_mass(*obj);
  if (!(Im > 0.0)) return -2;
  const int nd = 6 + hand->n_links - 1;
  const int nt = set_threads(n_threads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int b = 0; b < B; ++b) {
    std::vector<double> qq(q + static_cast<size_t>(b) * nd, q + static_cast<size_t>(b + 1) * nd);
    double L0, t4[4];
    Trace t0;
    candidate_step(*hand, *obj, Im, *prm, qq.data(), L0, t4, &t0);
    for (int j = 0; j < nd; ++j) {
      const double q0 = qq[j];
      double Lp, Lm;
      Trace tp, tm;
      qq[j] = q0 + fd_h;
      candidate_step(*hand, *obj, Im, *prm, qq.data(), Lp, t4, &tp);
      qq[j] = q0 - fd_h;
      candidate_step(*hand, *obj, Im, *prm, qq.data(), Lm, t4, &tm);
      qq[j] = q0;
      grad[static_cast<size_t>(b) * nd + j] = (Lp - Lm) / (2.0 * fd_h);
      if (excluded)
        excluded[static_cast<size_t>(b) * nd + j] = (tp.signature != t0.signature) || (tm.signature != t0.signature);
    }
  }
  return 0;
}

// Adam (Kingma & Ba): bias-corrected first and second moments, t >= 1.
int oracle_adam(int n, double* q, double* m, double* v, const double* g, int t, double lr, double b1, double b2,
                double eps) {
  if (n < 0 || t < 1 || (n > 0 && (!q || !m || !v || !g))) return -1;
  const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    q[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
  return 0;
}

int oracle_rank(int B, const double* loss, int* rank) {
  if (B < 0 || (B > 0 && (!loss || !rank))) return -1;
  std::vector<int> idx(B);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return loss[a] < loss[b]; });
  std::copy(idx.begin(), idx.end(), rank);
  return 0;
}

// Post-synthesis metrics (Sec. V-A). The paper names contact area and
// intersection volume without formulas; read here as integrals over the
// hand: CA(tau) = area of the hand surface whose signed distance to the
// object is below tau (penetrating surface is in contact), IV = volume of the
// hand whose signed distance is below 0, each estimated by the caller's
// weighted samples placed by forward kinematics at the candidate's q.
int oracle_evaluate(const ohand* hand, const oobject* obj, int B, const double* q, const oeval* ev, int n_thr,
                    const double* thr, double delta, double* out, double* slack, int n_threads) {
  if (!valid_hand(hand) || !valid_obj(obj) || !ev || B < 0 || n_thr < 0 || (B > 0 && (!q || !out)) ||
      (n_thr > 0 && !thr) || ev->n_surface < 0 || ev->n_volume < 0 || !(delta >= 0.0))
    return -1;
  if ((ev->n_surface > 0 && (!ev->surface_link || !ev->surface_local || !ev->surface_area)) ||
      (ev->n_volume > 0 && (!ev->volume_link || !ev->volume_local || !ev->volume_weight)))
    return -1;
  for (int i = 0; i < ev->n_surface; ++i)
    if (ev->surface_link[i] < 0 || ev->surface_link[i] >= hand->n_links) return -1;
  for (int i = 0; i < ev->n_volume; ++i)
    if (ev->volume_link[i] < 0 || ev->volume_link[i] >= hand->n_links) return -1;
  const int nd = 6 + hand->n_links - 1, M = n_thr + 1;
  const int nt = set_threads(n_threads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int b = 0; b < B; ++b) {
    const double* qb = q + static_cast<size_t>(b) * nd;
    double* o = out + static_cast<size_t>(b) * M;
    double* s = slack ? slack + static_cast<size_t>(b) * M : nullptr;
    for (int t = 0; t < M; ++t) {
      o[t] = 0.0;
      if (s) s[t] = 0.0;
    }
    bool finite = true;
    for (int j = 0; j < nd; ++j) finite = finite && std::isfinite(qb[j]);
    if (!finite) {
      for (int t = 0; t < M; ++t) o[t] = std::nan("");
      continue;
    }
    std::vector<Xf<double>> T;
    forward_kinematics(*hand, qb, T);
    auto phi_at = [&](int link, const double* local) {
      double p[3], n3[3], phi;
      apply_xf(T[link], local, p);
      sample_object(*obj, p, phi, n3, nullptr);
      return phi;
    };
    for (int i = 0; i < ev->n_surface; ++i) {
      const double phi = phi_at(ev->surface_link[i], ev->surface_local + 3 * i);
      const double a = ev->surface_area[i];
      for (int t = 0; t < n_thr; ++t) {
        if (phi < thr[t]) o[t] += a;
        if (s && std::fabs(phi - thr[t]) < delta) s[t] += a;
      }
    }
    for (int i = 0; i < ev->n_volume; ++i) {
      const double phi = phi_at(ev->volume_link[i], ev->volume_local + 3 * i);
      const double v = ev->volume_weight[i];
      if (phi < 0.0) o[n_thr] += v;
      if (s && std::fabs(phi) < delta) s[n_thr] += v;
    }
  }
  return 0;
}

// Top-k selection behind the paper's top-10 figures (Sec. V-A): the paper
// ranks by the epsilon metric; here the caller supplies the key.
int oracle_select_top(int B, const double* key, int higher_is_better, int k, int M, const double* metrics,
                      int* top, double* mean) {
  if (B < 0 || k < 0 || k > B || M < 0 || (B > 0 && !key) || (k > 0 && !top) || (M > 0 && k > 0 && (!metrics || !mean)))
    return -1;
  auto better = [&](int a, int b) {
    const bool na = std::isnan(key[a]), nb = std::isnan(key[b]);
    if (na || nb) return !na && nb;
    return higher_is_better ? key[a] > key[b] : key[a] < key[b];
  };
  std::vector<int> idx(B);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), better);
  for (int j = 0; j < k; ++j) top[j] = idx[j];
  for (int m = 0; m < M && k > 0; ++m) {
    double sum = 0.0;
    for (int j = 0; j < k; ++j) sum += metrics[static_cast<size_t>(top[j]) * M + m];
    mean[m] = sum / k;
  }
  return 0;
}

int oracle_optimize(const ohand* hand, const oobject* obj, const oparams* prm, int B, double* q, int T, double r0,
                    double lr, double b1, double b2, double eps, int use_gd, double* final_loss, double* final_terms,
                    int* rank, double* loss_hist, int n_threads) {
  if (!valid_hand(hand) || !valid_obj(obj) || !prm || B < 0 || T < 1 || (B > 0 && !q)) return -1;
  const int nd = 6 + hand->n_links - 1;
  std::vector<double> m(static_cast<size_t>(B) * nd, 0.0), v(static_cast<size_t>(B) * nd, 0.0);
  std::vector<double> g(static_cast<size_t>(B) * nd), L(B);
  oparams P = *prm;
  for (int t = 0; t < T; ++t) {
    // linear dilation schedule down to 0 at the last step (Sec. III-B)
    P.r_dil = (T > 1) ? r0 * (1.0 - static_cast<double>(t) / (T - 1)) : 0.0;
    int rc = oracle_step(hand, obj, &P, B, q, L.data(), nullptr, g.data(), nullptr, n_threads);
    if (rc) return rc;
    if (loss_hist) std::copy(L.begin(), L.end(), loss_hist + static_cast<size_t>(t) * B);
    if (use_gd) {
      for (size_t i = 0; i < g.size(); ++i) q[i] -= lr * g[i];
    } else {
      oracle_adam(B * nd, q, m.data(), v.data(), g.data(), t + 1, lr, b1, b2, eps);
    }
  }
  P.r_dil = 0.0;
  std::vector<double> terms(4 * static_cast<size_t>(B));
  int rc = oracle_step(hand, obj, &P, B, q, L.data(), terms.data(), nullptr, nullptr, n_threads);
  if (rc) return rc;
  if (final_loss) std::copy(L.begin(), L.end(), final_loss);
  if (final_terms) std::copy(terms.begin(), terms.end(), final_terms);
  if (rank) oracle_rank(B, L.data(), rank);
  return 0;
}

}  // extern "C"
