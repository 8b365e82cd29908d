// Device side of the mesh object (Sec. III-B): the Phong signed distance of
// a closed triangle mesh, queried through its bounding-volume hierarchy.
// Shared by the mesh kernels and the evaluation kernels.
#pragma once

#include "device_common.h"
#include "internal.h"

namespace grasp {
namespace meshdev {

using namespace dev;

struct TriPoint {
  V3 x;          // closest point
  float w0, w1, w2;  // its barycentric weights
  int feature;   // 0 interior, 1..3 vertex a, b, c, 4..6 edge ab, bc, ca
};

// Closest point of triangle (a, b, c) to p by region tests on the dot
// products of p's offsets with the edges.
__device__ __forceinline__ TriPoint closest_on_tri(V3 a, V3 b, V3 c, V3 p) {
  TriPoint t;
  const V3 ab = b - a, ac = c - a, ap = p - a;
  const float d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0f && d2 <= 0.0f) {
    t.x = a; t.w0 = 1.0f; t.w1 = 0.0f; t.w2 = 0.0f; t.feature = 1;
    return t;
  }
  const V3 bp = p - b;
  const float d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0f && d4 <= d3) {
    t.x = b; t.w0 = 0.0f; t.w1 = 1.0f; t.w2 = 0.0f; t.feature = 2;
    return t;
  }
  const float vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
    const float v = d1 / (d1 - d3);
    t.x = a + v * ab; t.w0 = 1.0f - v; t.w1 = v; t.w2 = 0.0f; t.feature = 4;
    return t;
  }
  const V3 cp = p - c;
  const float d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0f && d5 <= d6) {
    t.x = c; t.w0 = 0.0f; t.w1 = 0.0f; t.w2 = 1.0f; t.feature = 3;
    return t;
  }
  const float vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
    const float w = d2 / (d2 - d6);
    t.x = a + w * ac; t.w0 = 1.0f - w; t.w1 = 0.0f; t.w2 = w; t.feature = 6;
    return t;
  }
  const float va = d3 * d6 - d5 * d4;
  if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {
    const float w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    t.x = b + w * (c - b); t.w0 = 0.0f; t.w1 = 1.0f - w; t.w2 = w; t.feature = 5;
    return t;
  }
  const float den = 1.0f / (va + vb + vc);
  const float v = vb * den, w = vc * den;
  t.x = a + v * ab + w * ac; t.w0 = 1.0f - v - w; t.w1 = v; t.w2 = w; t.feature = 0;
  return t;
}

__device__ __forceinline__ V3 ld3(const float4 q) { return v3(q.x, q.y, q.z); }

// r - r* for the closest point t of triangle (a, b, c), taken from r's
// offsets (the plane offset along the unit face normal fn on the interior,
// the part across the edge's line on an edge) rather than as r minus the
// reconstructed closest point, whose micrometre-scale in-plane rounding would
// tilt the direction where r is close to the face. h: the plane offset
// (interior), ax: fn (interior), the edge's unit direction (edge) or 0.
__device__ __forceinline__ V3 offset_from_feature(const TriPoint& t, V3 a, V3 b, V3 c, V3 p, V3 fn, float& h, V3& ax) {
  h = 0.0f;
  if (t.feature == 0) {
    ax = fn;
    h = dot(p - a, fn);
    return h * fn;
  }
  if (t.feature >= 4) {
    const V3 e0 = t.feature == 4 ? a : (t.feature == 5 ? b : c);
    const V3 e = t.feature == 4 ? b - a : (t.feature == 5 ? c - b : a - c);
    ax = rsq(dot(e, e)) * e;
    const V3 o = p - e0;
    return o - dot(o, ax) * ax;
  }
  ax = v3(0.0f, 0.0f, 0.0f);
  return p - t.x;
}

// Squared distance from p to the box [lo, hi].
__device__ __forceinline__ float box_d2(float4 lo, float4 hi, V3 p) {
  const float dx = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.0f);
  const float dy = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.0f);
  const float dz = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.0f);
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Relative width of the band in which two squared distances are taken as
// equal: a few units in the last place of d^2 plus what the closest point's
// own rounding adds.
constexpr float kTieBand = 0x1p-19f;

// Nearest triangle to p: its index (-1 when p is not finite) and squared
// distance. A face whose closest point lies on an edge or vertex it shares
// with a neighbour that holds p's projection in its interior is never nearer
// than that neighbour, but in FP32 the two squared distances agree whenever
// the offset between the points is below about sqrt(ulp(d^2)) (micrometres
// at centimetres); within kTieBand the lower-dimensional region loses
// (interior before edge before vertex), which is the true order for shared
// features. The stack holds at most one entry per level of the hierarchy,
// whose depth the loader keeps below kMeshStack.
__device__ __forceinline__ int nearest_triangle(const MeshView& M, V3 p, float& best) {
  int stack[kMeshStack];
  int sp = 0;
  int node = 0;
  int bestf = -1;
  int brank = 3;
  best = INFINITY;
  float reach = INFINITY;  // best widened by the band: boxes beyond it cannot hold a tie
  if (!(box_d2(M.nodes[0], M.nodes[1], p) < reach)) return -1;
  for (;;) {
    const float4 lo = M.nodes[2 * node], hi = M.nodes[2 * node + 1];
    const int a = __float_as_int(lo.w), cnt = __float_as_int(hi.w);
    bool descend = false;
    if (cnt > 0) {
      for (int f = a; f < a + cnt; ++f) {
        const TriPoint t = closest_on_tri(ld3(M.tri[3 * f]), ld3(M.tri[3 * f + 1]), ld3(M.tri[3 * f + 2]), p);
        const V3 d = p - t.x;
        const float d2 = dot(d, d);
        const int rank = t.feature == 0 ? 0 : (t.feature >= 4 ? 1 : 2);
        const float band = kTieBand * best;
        const bool take = rank < brank ? d2 <= best + band : (rank == brank ? d2 < best : d2 < best - band);
        if (take) {
          best = d2;
          bestf = f;
          brank = rank;
          reach = fmaf(kTieBand, d2, d2);
        }
      }
    } else {
      const int l = node + 1, r = a;
      const float dl = box_d2(M.nodes[2 * l], M.nodes[2 * l + 1], p);
      const float dr = box_d2(M.nodes[2 * r], M.nodes[2 * r + 1], p);
      const bool left_first = dl <= dr;
      const int nn = left_first ? l : r, nf = left_first ? r : l;
      const float dn = left_first ? dl : dr, df = left_first ? dr : dl;
      if (df <= reach) stack[sp++] = nf;
      if (dn <= reach) {
        node = nn;
        descend = true;
      }
    }
    if (descend) continue;
    bool found = false;
    while (sp > 0) {
      node = stack[--sp];
      if (box_d2(M.nodes[2 * node], M.nodes[2 * node + 1], p) <= reach) {
        found = true;
        break;
      }
    }
    if (!found) break;
  }
  return bestf;
}

// nearest_triangle for the lanes of one wave at once, called by every lane of
// the wave together (active: the lane wants its point's face; the others
// return -1). The wave walks one path, the union of what its lanes need: a
// node is entered when some lane's reach covers its box, and every lane tests
// the faces of each leaf entered, keeping its own best under the same tie
// rule. The node and face records are read at a wave-uniform index. The
// stack holds one entry per level in one register across the lanes (entry k
// in lane k): the loader keeps the depth below kMeshStack, which fits a wave.
static_assert(kMeshStack <= kWave, "the wave's stack has one entry per lane");
__device__ __forceinline__ int nearest_triangle_wave(const MeshView& M, V3 p, float& best, bool active) {
  const int lane = __lane_id();
  int stk = 0;
  int sp = 0;
  int bestf = -1;
  int brank = 3;
  best = INFINITY;
  // as in nearest_triangle, a point whose distance to the root box is not
  // below infinity (not finite, or too far for FP32) gets -1; such lanes and
  // the inactive ones never reach a box (box_d2 >= 0) and take no face
  const bool live = active && box_d2(M.nodes[0], M.nodes[1], p) < INFINITY;
  float reach = live ? INFINITY : -1.0f;
  if (__builtin_amdgcn_ballot_w64(live) == 0) return -1;
  int node = 0;
  for (;;) {
    const float4 lo = M.nodes[2 * node], hi = M.nodes[2 * node + 1];
    const int a = __float_as_int(lo.w), cnt = __float_as_int(hi.w);
    if (cnt > 0) {
      for (int f = a; f < a + cnt; ++f) {
        const TriPoint t = closest_on_tri(ld3(M.tri[3 * f]), ld3(M.tri[3 * f + 1]), ld3(M.tri[3 * f + 2]), p);
        const V3 d = p - t.x;
        const float d2 = dot(d, d);
        const int rank = t.feature == 0 ? 0 : (t.feature >= 4 ? 1 : 2);
        const float band = kTieBand * best;
        const bool take =
            live && (rank < brank ? d2 <= best + band : (rank == brank ? d2 < best : d2 < best - band));
        if (take) {
          best = d2;
          bestf = f;
          brank = rank;
          reach = fmaf(kTieBand, d2, d2);
        }
      }
    } else {
      const int l = node + 1, r = a;
      const float dl = box_d2(M.nodes[2 * l], M.nodes[2 * l + 1], p);
      const float dr = box_d2(M.nodes[2 * r], M.nodes[2 * r + 1], p);
      const uint64_t bl = __builtin_amdgcn_ballot_w64(dl <= reach);
      const uint64_t br = __builtin_amdgcn_ballot_w64(dr <= reach);
      if (bl != 0 && br != 0) {
        // nearer child first by the lanes' majority
        const int nl = __builtin_popcountll(__builtin_amdgcn_ballot_w64(dl <= reach && dl <= dr));
        const int nr = __builtin_popcountll(__builtin_amdgcn_ballot_w64(dr <= reach && dr < dl));
        const bool left_first = nl >= nr;
        stk = lane == sp ? (left_first ? r : l) : stk;
        ++sp;
        node = left_first ? l : r;
        continue;
      }
      if (bl != 0 || br != 0) {
        node = bl != 0 ? l : r;
        continue;
      }
    }
    bool found = false;
    while (sp > 0) {
      --sp;
      node = __builtin_amdgcn_readlane(stk, sp);
      if (__builtin_amdgcn_ballot_w64(box_d2(M.nodes[2 * node], M.nodes[2 * node + 1], p) <= reach) != 0) {
        found = true;
        break;
      }
    }
    if (!found) break;
  }
  return bestf;
}

// Phong signed distance and its stated gradient at p.
// (mesh_sdf_face: the same given p's nearest face f from either walk.)
__device__ __forceinline__ void mesh_sdf_face(const MeshView& M, int f, V3 p, float& rho, V3& g) {
  if (f < 0) {
    rho = __builtin_nanf("");
    g = v3(rho, rho, rho);
    return;
  }
  const V3 a = ld3(M.tri[3 * f]), b = ld3(M.tri[3 * f + 1]), c = ld3(M.tri[3 * f + 2]);
  const TriPoint t = closest_on_tri(a, b, c, p);
  const float* I = M.info + static_cast<size_t>(f) * kMeshInfo;
  auto I3 = [&](int k) { return v3(I[3 * k], I[3 * k + 1], I[3 * k + 2]); };
  // pseudonormal of the closest feature: [3] face, [4..6] edges ab, bc, ca, [7..9] vertices a, b, c
  const int slot = t.feature == 0 ? 3 : (t.feature <= 3 ? 6 + t.feature : t.feature);
  float h;
  V3 ax;
  const V3 rr = offset_from_feature(t, a, b, c, p, I3(3), h, ax);
  const float s = dot(rr, I3(slot)) >= 0.0f ? 1.0f : -1.0f;
  // curved point q = r* - alpha pull: r* pulled towards the tangent planes
  // of the three vertices
  const float wv[3] = {t.w0, t.w1, t.w2};
  const V3 vv[3] = {a, b, c};
  V3 pull = v3(0.0f, 0.0f, 0.0f);
  for (int k = 0; k < 3; ++k) {
    const V3 nk = I3(k);
    pull = pull + (wv[k] * dot(t.x - vv[k], nk)) * nk;
  }
  const V3 d = rr + M.alpha * pull;
  const float dist = sqrtf(dot(d, d));
  rho = s * dist;
  g = dist > 0.0f ? (1.0f / rho) * d : I3(3);
}

__device__ __forceinline__ void mesh_sdf(const MeshView& M, V3 p, float& rho, V3& g) {
  float best;
  mesh_sdf_face(M, nearest_triangle(M, p, best), p, rho, g);
}

// The Phong distance at a sample of the grasp step, with what its adjoint
// needs. With q the Phong point, n = (r - q) / rho the stated normal (the
// constraint's direction) and J_q = dq/dr:
//   grad rho = (I - J_q)^T n                      (the exact gradient of rho)
//   (dn/dr)^T v = ((I - J_q)^T v - (n . v) grad rho) / rho.
// J_q = (dq/dr*) (dr*/dr): r* moves with r as the projection onto the face
// plane (interior), onto the edge's line (edge) or not at all (vertex), and
//   dq/dr* = I - alpha sum_k (n_k h_k grad(w_k)^T + w_k n_k n_k^T),
// h_k = (r* - v_k) . n_k, w_k the barycentric weights of r* on the face.
struct MeshSample {
  float rho;
  V3 n;           // stated normal
  V3 grad;        // exact gradient of rho
  float inv_rho;  // 1 / rho (0 on the Phong surface, where n is the face normal)
  int region;     // 0 face interior, 1 edge, 2 vertex
  V3 ax;          // face unit normal (interior) or edge unit direction (edge)
  V3 nk[3];       // vertex normals
  V3 gw[3];       // barycentric gradients
  float hk[3], wk[3];
  float h;        // interior: signed offset of r from the face plane along ax
  V3 pull;        // sum_k w_k h_k n_k, so that r - q = (r - r*) + alpha pull
};

// J_q^T v for the sample's closest feature.
__device__ __forceinline__ V3 mesh_jq_t(const MeshSample& s, float alpha, V3 v) {
  V3 out = v;
  for (int k = 0; k < 3; ++k) {
    const float nv = dot(s.nk[k], v);
    out = out - (alpha * s.hk[k] * nv) * s.gw[k] - (alpha * s.wk[k] * nv) * s.nk[k];
  }
  if (s.region == 0) return out - dot(s.ax, out) * s.ax;
  if (s.region == 1) return dot(s.ax, out) * s.ax;
  return v3(0.0f, 0.0f, 0.0f);
}

// (dn/dr)^T v = (I - J_q)^T P v / rho, P = I - n n^T. On a face interior
// I - J_q^T = f f^T + alpha T A^T (f the face normal, T = I - f f^T, A^T the
// Phong part of J_q^T), and with r - q = h f + alpha pull the component
// f . P v = alpha ((f.v)(h pf + alpha |pull|^2) - (pull.v)(h + alpha pf)) / rho^2,
// pf = pull . f: written so, it vanishes exactly on a flat face (alpha = 0)
// instead of leaving FP32 noise divided by rho, which is large where r is
// micrometres from the surface. Edges and vertices turn n at the rate 1/rho
// in exact arithmetic too and keep the plain form.
__device__ __forceinline__ V3 mesh_ngrad_t(const MeshSample& s, float alpha, V3 v) {
  if (s.inv_rho == 0.0f) return v3(0.0f, 0.0f, 0.0f);
  if (s.region != 0) return s.inv_rho * ((v - mesh_jq_t(s, alpha, v)) - dot(s.n, v) * s.grad);
  const V3 f = s.ax;
  const V3 pv = v - dot(s.n, v) * s.n;
  const float pf = dot(s.pull, f);
  const float fpv = alpha * (dot(f, v) * (s.h * pf + alpha * dot(s.pull, s.pull)) - dot(s.pull, v) * (s.h + alpha * pf)) *
                    (s.inv_rho * s.inv_rho);
  V3 at = v3(0.0f, 0.0f, 0.0f);
  for (int k = 0; k < 3; ++k) {
    const float nv = dot(s.nk[k], pv);
    at = at + (s.hk[k] * nv) * s.gw[k] + (s.wk[k] * nv) * s.nk[k];
  }
  at = alpha * (at - dot(f, at) * f);
  return s.inv_rho * (fpv * f + at);
}

// The sample at p given its nearest face f (from nearest_triangle; < 0: p
// not finite).
__device__ __forceinline__ void mesh_sample_face(const MeshView& M, int f, V3 p, MeshSample& s) {
  if (f < 0) {
    const float nan = __builtin_nanf("");
    s.rho = nan;
    s.n = s.grad = s.ax = v3(nan, nan, nan);
    s.inv_rho = 0.0f;
    s.region = 2;
    for (int k = 0; k < 3; ++k) {
      s.nk[k] = s.gw[k] = v3(0.0f, 0.0f, 0.0f);
      s.hk[k] = s.wk[k] = 0.0f;
    }
    return;
  }
  const V3 a = ld3(M.tri[3 * f]), b = ld3(M.tri[3 * f + 1]), c = ld3(M.tri[3 * f + 2]);
  const TriPoint t = closest_on_tri(a, b, c, p);
  const float* I = M.info + static_cast<size_t>(f) * kMeshInfo;
  auto I3 = [&](int k) { return v3(I[3 * k], I[3 * k + 1], I[3 * k + 2]); };
  const int slot = t.feature == 0 ? 3 : (t.feature <= 3 ? 6 + t.feature : t.feature);
  const V3 vv[3] = {a, b, c};
  s.wk[0] = t.w0;
  s.wk[1] = t.w1;
  s.wk[2] = t.w2;
  V3 pull = v3(0.0f, 0.0f, 0.0f);
  for (int k = 0; k < 3; ++k) {
    s.nk[k] = I3(k);
    s.hk[k] = dot(t.x - vv[k], s.nk[k]);
    pull = pull + (s.wk[k] * s.hk[k]) * s.nk[k];
  }
  s.pull = pull;
  // barycentric gradients on the face: grad w_a = N x (c - b) / |N|^2, ...
  const V3 N = cross(b - a, c - a);
  const float inn = 1.0f / dot(N, N);
  s.gw[0] = inn * cross(N, c - b);
  s.gw[1] = inn * cross(N, a - c);
  s.gw[2] = inn * cross(N, b - a);
  s.region = t.feature == 0 ? 0 : (t.feature >= 4 ? 1 : 2);
  const V3 rr = offset_from_feature(t, a, b, c, p, I3(3), s.h, s.ax);
  const float sg = dot(rr, I3(slot)) >= 0.0f ? 1.0f : -1.0f;
  const V3 d = rr + M.alpha * pull;
  const float dist = sqrtf(dot(d, d));
  if (dist > 0.0f) {
    s.rho = sg * dist;
    s.inv_rho = 1.0f / s.rho;
    s.n = s.inv_rho * d;
    s.grad = s.n - mesh_jq_t(s, M.alpha, s.n);
  } else {
    s.rho = 0.0f;
    s.inv_rho = 0.0f;
    s.n = I3(3);
    s.grad = s.n;
  }
}

__device__ __forceinline__ void mesh_sample(const MeshView& M, V3 p, MeshSample& s) {
  float best;
  mesh_sample_face(M, nearest_triangle(M, p, best), p, s);
}

// mesh_sample through nearest_triangle_wave: every lane of the wave calls it.
__device__ __forceinline__ void mesh_sample_wave(const MeshView& M, V3 p, MeshSample& s) {
  float best;
  mesh_sample_face(M, nearest_triangle_wave(M, p, best, true), p, s);
}

}  // namespace meshdev
}  // namespace grasp
