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

// Squared distance from p to the box [lo, hi].
__device__ __forceinline__ float box_d2(float4 lo, float4 hi, V3 p) {
  const float dx = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.0f);
  const float dy = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.0f);
  const float dz = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.0f);
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Nearest triangle to p: its index (-1 when p is not finite) and squared
// distance. The stack holds at most one entry per level of the hierarchy,
// whose depth the loader keeps below kMeshStack.
__device__ __forceinline__ int nearest_triangle(const MeshView& M, V3 p, float& best) {
  int stack[kMeshStack];
  int sp = 0;
  int node = 0;
  int bestf = -1;
  best = INFINITY;
  if (!(box_d2(M.nodes[0], M.nodes[1], p) < best)) return -1;
  for (;;) {
    const float4 lo = M.nodes[2 * node], hi = M.nodes[2 * node + 1];
    const int a = __float_as_int(lo.w), cnt = __float_as_int(hi.w);
    bool descend = false;
    if (cnt > 0) {
      for (int f = a; f < a + cnt; ++f) {
        const TriPoint t = closest_on_tri(ld3(M.tri[3 * f]), ld3(M.tri[3 * f + 1]), ld3(M.tri[3 * f + 2]), p);
        const V3 d = p - t.x;
        const float d2 = dot(d, d);
        if (d2 < best) {
          best = d2;
          bestf = f;
        }
      }
    } else {
      const int l = node + 1, r = a;
      const float dl = box_d2(M.nodes[2 * l], M.nodes[2 * l + 1], p);
      const float dr = box_d2(M.nodes[2 * r], M.nodes[2 * r + 1], p);
      const bool left_first = dl <= dr;
      const int nn = left_first ? l : r, nf = left_first ? r : l;
      const float dn = left_first ? dl : dr, df = left_first ? dr : dl;
      if (df < best) stack[sp++] = nf;
      if (dn < best) {
        node = nn;
        descend = true;
      }
    }
    if (descend) continue;
    bool found = false;
    while (sp > 0) {
      node = stack[--sp];
      if (box_d2(M.nodes[2 * node], M.nodes[2 * node + 1], p) < best) {
        found = true;
        break;
      }
    }
    if (!found) break;
  }
  return bestf;
}

// Phong signed distance and its stated gradient at p.
__device__ __forceinline__ void mesh_sdf(const MeshView& M, V3 p, float& rho, V3& g) {
  float best;
  const int f = nearest_triangle(M, p, best);
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
  const float s = dot(p - t.x, I3(slot)) >= 0.0f ? 1.0f : -1.0f;
  // curved point: r* pulled towards the tangent planes of the three vertices
  const float wv[3] = {t.w0, t.w1, t.w2};
  const V3 vv[3] = {a, b, c};
  V3 pull = v3(0.0f, 0.0f, 0.0f);
  for (int k = 0; k < 3; ++k) {
    const V3 nk = I3(k);
    pull = pull + (wv[k] * dot(t.x - vv[k], nk)) * nk;
  }
  const V3 q = t.x - M.alpha * pull;
  const V3 d = p - q;
  const float dist = sqrtf(dot(d, d));
  rho = s * dist;
  g = dist > 0.0f ? (1.0f / rho) * d : I3(3);
}

}  // namespace meshdev
}  // namespace grasp
