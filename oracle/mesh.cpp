// FP64 oracle of the mesh object's Phong signed distance (Sec. III-B).
//
// TEST INFRASTRUCTURE ONLY, like the rest of the oracle: plain, slow and
// written to be checked by eye. Brute force over every triangle; no
// acceleration structure.
//
// phi(r) = s(r) |r - r*| with r* the closest point of the triangle mesh and
// s = -1 inside the closed mesh, +1 outside. The sign comes from the
// generalized winding number (the solid angle the mesh subtends at r over
// 4 pi: 1 inside a closed outward-oriented mesh, 0 outside); the paper casts a
// ray, which decides the same inside/outside question.
//
// The Phong distance replaces r* by a point of the curved (Phong) triangle:
// with r* = u v_i + v v_j + w v_k and psi_b(x) the projection of x onto the
// plane through v_b with normal n_b (the vertex normal),
//   p = (1 - alpha) r* + alpha (u psi_i(r*) + v psi_j(r*) + w psi_k(r*)),
//   rho(r) = s(r) |r - p|,   grad rho = (r - p) / rho
// (the gradient the paper states; at rho = 0 the face normal).

#include <cmath>

#include "oracle_api.h"

namespace {

struct D3 {
  double x, y, z;
};
D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(D3 a) { return std::sqrt(dot(a, a)); }
D3 load(const double* p) { return {p[0], p[1], p[2]}; }

// Closest point of triangle (a, b, c) to r, with its barycentric weights
// (wa, wb, wc). The point is the minimizer of |r - x| over the triangle: the
// projection onto the plane when it falls inside, otherwise the closest point
// of the nearest edge segment (or a vertex). Each edge is clamped to its
// segment; the best of the three candidates wins.
D3 closest_on_triangle(D3 a, D3 b, D3 c, D3 r, double bary[3]) {
  const D3 n = cross(b - a, c - a);
  const double nn = dot(n, n);
  // projection onto the plane and its barycentric coordinates
  const D3 x = r - (dot(r - a, n) / nn) * n;
  const double wa = dot(cross(c - b, x - b), n) / nn;
  const double wb = dot(cross(a - c, x - c), n) / nn;
  const double wc = 1.0 - wa - wb;
  if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
    bary[0] = wa;
    bary[1] = wb;
    bary[2] = wc;
    return x;
  }
  // nearest point of each edge segment p0 + t (p1 - p0), t in [0, 1]
  const D3 P[3] = {a, b, c};
  double best = INFINITY;
  D3 out{0, 0, 0};
  for (int e = 0; e < 3; ++e) {
    const int i0 = e, i1 = (e + 1) % 3;
    const D3 d = P[i1] - P[i0];
    double t = dot(r - P[i0], d) / dot(d, d);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const D3 y = P[i0] + t * d;
    const double dist = norm(r - y);
    if (dist < best) {
      best = dist;
      out = y;
      bary[0] = bary[1] = bary[2] = 0.0;
      bary[i0] = 1.0 - t;
      bary[i1] = t;
    }
  }
  return out;
}

// Signed solid angle of triangle (a, b, c) seen from r (positive when the
// triangle winds counter-clockwise seen from r's side opposite its normal,
// i.e. when r is behind an outward face), by the half-angle tangent formula
// of Van Oosterom and Strackee.
double solid_angle(D3 a, D3 b, D3 c, D3 r) {
  const D3 A = a - r, B = b - r, C = c - r;
  const double la = norm(A), lb = norm(B), lc = norm(C);
  const double num = dot(A, cross(B, C));
  const double den = la * lb * lc + dot(A, B) * lc + dot(A, C) * lb + dot(B, C) * la;
  return 2.0 * std::atan2(num, den);
}

// Phong point of face f's point y with barycentric weights w: the blend of
// y and its projections onto the tangent planes of the face's vertices.
D3 phong_point(const omesh* m, int f, D3 y, const double w[3]) {
  const int* t = m->faces + 3 * f;
  D3 curved{0, 0, 0};
  for (int j = 0; j < 3; ++j) {
    const D3 v = load(m->vertices + 3 * t[j]);
    const D3 nv = load(m->normals + 3 * t[j]);
    curved = curved + w[j] * (y - dot(y - v, nv) * nv);
  }
  return (1.0 - m->alpha) * y + m->alpha * curved;
}

}  // namespace

extern "C" {

double oracle_winding_number(const omesh* m, const double* r) {
  if (!m || !r) return NAN;
  const D3 x = load(r);
  double s = 0.0;
  for (int f = 0; f < m->n_faces; ++f) {
    const int* t = m->faces + 3 * f;
    s += solid_angle(load(m->vertices + 3 * t[0]), load(m->vertices + 3 * t[1]), load(m->vertices + 3 * t[2]), x);
  }
  return s / (4.0 * M_PI);
}

int oracle_closest_on_triangle(const double* a, const double* b, const double* c, const double* r, double* out,
                               double* bary) {
  if (!a || !b || !c || !r || !out || !bary) return -1;
  const D3 x = closest_on_triangle(load(a), load(b), load(c), load(r), bary);
  out[0] = x.x;
  out[1] = x.y;
  out[2] = x.z;
  return 0;
}

int oracle_mesh_sdf(const omesh* m, int n, const double* r, double* rho, double* grad, double* closest,
                    int* face, double* dist_flat, double* gap, double* spread) {
  if (!m || n < 0 || (n > 0 && (!r || !rho)) || m->n_faces < 1) return -1;
  for (int k = 0; k < n; ++k) {
    const D3 x = load(r + 3 * k);
    double best = INFINITY, bb[3] = {0, 0, 0};
    int bf = -1;
    D3 bx{0, 0, 0};
    for (int f = 0; f < m->n_faces; ++f) {
      const int* t = m->faces + 3 * f;
      double w[3];
      const D3 y = closest_on_triangle(load(m->vertices + 3 * t[0]), load(m->vertices + 3 * t[1]),
                                       load(m->vertices + 3 * t[2]), x, w);
      const double d = norm(x - y);
      if (d < best) {
        best = d;
        bf = f;
        bx = y;
        bb[0] = w[0];
        bb[1] = w[1];
        bb[2] = w[2];
      }
    }
    // how much farther the nearest point of any face is when it is a
    // different point (faces sharing the closest edge or vertex give the same
    // point and the same Phong point); small where r is nearly equidistant
    // from two parts of the surface
    double second = INFINITY;
    for (int f = 0; f < m->n_faces; ++f) {
      const int* t = m->faces + 3 * f;
      double w[3];
      const D3 y = closest_on_triangle(load(m->vertices + 3 * t[0]), load(m->vertices + 3 * t[1]),
                                       load(m->vertices + 3 * t[2]), x, w);
      if (norm(y - bx) > 1e-9) second = std::fmin(second, norm(x - y));
    }
    const double s = oracle_winding_number(m, r + 3 * k) > 0.5 ? -1.0 : 1.0;
    // Phong point: blend of the flat closest point and its projections onto
    // the tangent planes of the face's three vertices
    const int* t = m->faces + 3 * bf;
    const D3 p = phong_point(m, bf, bx, bb);
    const double dist = norm(x - p);
    if (spread) {
      // faces whose flat distance is within single-precision resolution of
      // the best one: how far apart their Phong distances lie
      const double eps = 4e-7 * (best + norm(x));
      double sp = 0.0;
      for (int f = 0; f < m->n_faces; ++f) {
        const int* u = m->faces + 3 * f;
        double w[3];
        const D3 y = closest_on_triangle(load(m->vertices + 3 * u[0]), load(m->vertices + 3 * u[1]),
                                         load(m->vertices + 3 * u[2]), x, w);
        if (norm(x - y) <= best + eps) sp = std::fmax(sp, std::fabs(norm(x - phong_point(m, f, y, w)) - dist));
      }
      spread[k] = sp;
    }
    rho[k] = s * dist;
    if (grad) {
      D3 g;
      if (dist > 0.0) {
        g = (1.0 / rho[k]) * (x - p);
      } else {
        const D3 a = load(m->vertices + 3 * t[0]);
        const D3 fn = cross(load(m->vertices + 3 * t[1]) - a, load(m->vertices + 3 * t[2]) - a);
        g = (1.0 / norm(fn)) * fn;
      }
      grad[3 * k] = g.x;
      grad[3 * k + 1] = g.y;
      grad[3 * k + 2] = g.z;
    }
    if (closest) {
      closest[3 * k] = bx.x;
      closest[3 * k + 1] = bx.y;
      closest[3 * k + 2] = bx.z;
    }
    if (face) face[k] = bf;
    if (dist_flat) dist_flat[k] = best;
    if (gap) gap[k] = second - best;
  }
  return 0;
}

}  // extern "C"
