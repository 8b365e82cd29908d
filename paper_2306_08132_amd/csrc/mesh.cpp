// Mesh objects (Sec. III-B), host side: validation of a closed oriented
// triangle mesh, its pseudonormals, the bounding-volume hierarchy the query
// kernel walks, and the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>
#include <vector>

#include "grasp.h"
#include "context.h"
#include "internal.h"

using namespace grasp;

namespace {

using D3 = std::array<double, 3>;
D3 sub(const D3& a, const D3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
D3 add(const D3& a, const D3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
D3 scale(double s, const D3& a) { return {s * a[0], s * a[1], s * a[2]}; }
double dot(const D3& a, const D3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
D3 cross(const D3& a, const D3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const D3& a) { return std::sqrt(dot(a, a)); }
D3 unit(const D3& a) { return scale(1.0 / norm(a), a); }

struct Node {
  float lo[3], hi[3];
  int a = 0, count = 0;  // leaf: first face, count; internal: right child, 0
};

// Median split on the longest axis of the face centroids; leaves of at most
// four faces. Children of node k: k + 1 and Node::a (depth-first order).
struct Builder {
  const std::vector<std::array<float, 9>>& tv;  // face vertex positions
  std::vector<D3> centroid;
  std::vector<int> order;
  std::vector<Node> nodes;
  int max_depth = 0;

  explicit Builder(const std::vector<std::array<float, 9>>& t) : tv(t) {
    centroid.resize(t.size());
    for (size_t f = 0; f < t.size(); ++f)
      for (int k = 0; k < 3; ++k) centroid[f][k] = (double(t[f][k]) + t[f][3 + k] + t[f][6 + k]) / 3.0;
    order.resize(t.size());
    std::iota(order.begin(), order.end(), 0);
  }

  int build(int begin, int end, int depth) {
    max_depth = std::max(max_depth, depth);
    const int id = static_cast<int>(nodes.size());
    nodes.emplace_back();
    Node nd;
    for (int k = 0; k < 3; ++k) {
      nd.lo[k] = INFINITY;
      nd.hi[k] = -INFINITY;
    }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = begin; i < end; ++i) {
      const auto& t = tv[order[i]];
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) {
          nd.lo[k] = std::min(nd.lo[k], t[3 * v + k]);
          nd.hi[k] = std::max(nd.hi[k], t[3 * v + k]);
        }
      for (int k = 0; k < 3; ++k) {
        clo[k] = std::min(clo[k], centroid[order[i]][k]);
        chi[k] = std::max(chi[k], centroid[order[i]][k]);
      }
    }
    // leaves of up to 8 faces: against 4, fewer boxes tested per walk for the
    // same face tests (the mesh step 197 -> 178 ms, queries 4-9% faster; 2,
    // 12 and 16 were slower)
    if (end - begin <= 8) {
      nd.a = begin;
      nd.count = end - begin;
      nodes[id] = nd;
      return id;
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    const int mid = (begin + end) / 2;
    std::nth_element(order.begin() + begin, order.begin() + mid, order.begin() + end,
                     [&](int x, int y) { return centroid[x][axis] < centroid[y][axis]; });
    build(begin, mid, depth + 1);
    nd.a = build(mid, end, depth + 1);
    nd.count = 0;
    nodes[id] = nd;
    return id;
  }
};

float bits_as_float(int i) {
  float f;
  std::memcpy(&f, &i, sizeof f);
  return f;
}

DevMesh* find_mesh(grasp_ctx* ctx, grasp_mesh_id id) {
  auto it = ctx->meshes.find(id);
  return it == ctx->meshes.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

grasp_status grasp_load_mesh(grasp_ctx* ctx, const grasp_mesh_desc* d, grasp_mesh_id* out) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (!d || !out || !d->vertices || !d->faces) return fail(GRASP_EINVAL, "desc/out/vertices/faces is NULL");
  const int V = d->n_vertices, F = d->n_faces;
  if (V < 3 || V > (1 << 24)) return fail(GRASP_EINVAL, "n_vertices must be in [3, 2^24]");
  if (F < 4 || F > (1 << 22)) return fail(GRASP_EINVAL, "n_faces must be in [4, 2^22]");
  if (!(d->alpha >= 0.0f && d->alpha <= 1.0f)) return fail(GRASP_EINVAL, "alpha must be in [0, 1]");
  std::vector<D3> P(V);
  for (int i = 0; i < V; ++i)
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(d->vertices[3 * i + k])) return fail(GRASP_EINVAL, "vertex coordinates must be finite");
      P[i][k] = d->vertices[3 * i + k];
    }
  // faces, their unit normals and the angle of each corner
  std::vector<D3> fn(F);
  std::vector<std::array<double, 3>> corner(F);
  double volume = 0.0, max_edge = 0.0;
  for (int f = 0; f < F; ++f) {
    const int* t = d->faces + 3 * f;
    for (int j = 0; j < 3; ++j)
      if (t[j] < 0 || t[j] >= V) return fail(GRASP_EINVAL, "face index out of range");
    if (t[0] == t[1] || t[1] == t[2] || t[2] == t[0]) return fail(GRASP_EINVAL, "face repeats a vertex");
    const D3 n = cross(sub(P[t[1]], P[t[0]]), sub(P[t[2]], P[t[0]]));
    if (!(norm(n) > 0.0)) return fail(GRASP_EINVAL, "face of zero area");
    fn[f] = unit(n);
    volume += dot(P[t[0]], cross(P[t[1]], P[t[2]])) / 6.0;
    for (int j = 0; j < 3; ++j) max_edge = std::max(max_edge, norm(sub(P[t[(j + 1) % 3]], P[t[j]])));
    for (int j = 0; j < 3; ++j) {
      const D3 e1 = unit(sub(P[t[(j + 1) % 3]], P[t[j]])), e2 = unit(sub(P[t[(j + 2) % 3]], P[t[j]]));
      corner[f][j] = std::acos(std::max(-1.0, std::min(1.0, dot(e1, e2))));
    }
  }
  if (!(volume > 0.0)) return fail(GRASP_EINVAL, "mesh must enclose a positive volume (faces counter-clockwise from outside)");
  // every directed edge once, and its reverse exactly once: directed edges
  // as (u V + v, face) sorted by key
  std::vector<std::pair<uint64_t, int>> edges;
  edges.reserve(3 * static_cast<size_t>(F));
  auto key = [V](int u, int v) { return static_cast<uint64_t>(u) * static_cast<uint64_t>(V) + static_cast<uint64_t>(v); };
  for (int f = 0; f < F; ++f)
    for (int j = 0; j < 3; ++j) edges.emplace_back(key(d->faces[3 * f + j], d->faces[3 * f + (j + 1) % 3]), f);
  std::sort(edges.begin(), edges.end());
  for (size_t i = 1; i < edges.size(); ++i)
    if (edges[i].first == edges[i - 1].first) return fail(GRASP_EINVAL, "mesh is not consistently oriented");
  // the face across directed edge (u, v): the one holding (v, u), or -1
  auto across = [&](int u, int v) {
    const uint64_t k = key(v, u);
    const auto it = std::lower_bound(edges.begin(), edges.end(), std::make_pair(k, -1));
    return it != edges.end() && it->first == k ? it->second : -1;
  };
  for (const auto& e : edges)
    if (across(static_cast<int>(e.first / V), static_cast<int>(e.first % V)) < 0)
      return fail(GRASP_EINVAL, "mesh is not closed (an edge has one face)");
  // angle-weighted vertex pseudonormals
  std::vector<D3> vn(V, D3{0, 0, 0});
  for (int f = 0; f < F; ++f)
    for (int j = 0; j < 3; ++j) vn[d->faces[3 * f + j]] = add(vn[d->faces[3 * f + j]], scale(corner[f][j], fn[f]));
  for (int i = 0; i < V; ++i) {
    if (!(norm(vn[i]) > 0.0)) return fail(GRASP_EINVAL, "a vertex belongs to no face");
    vn[i] = unit(vn[i]);
  }
  std::vector<D3> phong(V);
  for (int i = 0; i < V; ++i) {
    if (d->normals) {
      D3 n{d->normals[3 * i], d->normals[3 * i + 1], d->normals[3 * i + 2]};
      if (!std::isfinite(n[0]) || !std::isfinite(n[1]) || !std::isfinite(n[2]) || !(norm(n) > 0.0))
        return fail(GRASP_EINVAL, "vertex normals must be finite and non-zero");
      phong[i] = unit(n);
    } else {
      phong[i] = vn[i];
    }
  }
  // hierarchy over the faces
  std::vector<std::array<float, 9>> tv(F);
  for (int f = 0; f < F; ++f)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) tv[f][3 * j + k] = d->vertices[3 * d->faces[3 * f + j] + k];
  Builder B(tv);
  B.build(0, F, 0);
  if (B.max_depth + 1 >= kMeshStack) return fail(GRASP_EINVAL, "mesh hierarchy too deep");
  // device records, faces in leaf order
  const size_t nn = B.nodes.size();
  std::vector<float4> hnodes(2 * nn), htri(3 * static_cast<size_t>(F));
  std::vector<float> hinfo(static_cast<size_t>(F) * kMeshInfo, 0.0f);
  for (size_t i = 0; i < nn; ++i) {
    const Node& n = B.nodes[i];
    hnodes[2 * i] = make_float4(n.lo[0], n.lo[1], n.lo[2], bits_as_float(n.a));
    hnodes[2 * i + 1] = make_float4(n.hi[0], n.hi[1], n.hi[2], bits_as_float(n.count));
  }
  for (int s = 0; s < F; ++s) {
    const int f = B.order[s];
    const int* t = d->faces + 3 * f;
    for (int j = 0; j < 3; ++j) htri[3 * s + j] = make_float4(tv[f][3 * j], tv[f][3 * j + 1], tv[f][3 * j + 2], 0.0f);
    float* I = hinfo.data() + static_cast<size_t>(s) * kMeshInfo;
    auto put = [&](int slot, const D3& v) {
      for (int k = 0; k < 3; ++k) I[3 * slot + k] = static_cast<float>(v[k]);
    };
    for (int j = 0; j < 3; ++j) put(j, phong[t[j]]);
    put(3, fn[f]);
    for (int j = 0; j < 3; ++j) {
      // edge (t[j], t[j+1]) and the face across it
      const int g = across(t[j], t[(j + 1) % 3]);
      put(4 + j, unit(add(fn[f], fn[g])));
      put(7 + j, vn[t[j]]);
    }
  }
  const size_t bn = round_up_bytes(hnodes.size() * sizeof(float4)), bt = round_up_bytes(htri.size() * sizeof(float4));
  const size_t bi = round_up_bytes(hinfo.size() * sizeof(float));
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(GRASP_EDEVICE, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(ctx->mu);
  void* blk = ctx->arena.alloc(bn + bt + bi);
  if (!blk) return fail(GRASP_ENOMEM, "arena full (mesh)");
  char* b = static_cast<char*>(blk);
  hipError_t e = hipMemcpy(b, hnodes.data(), hnodes.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b + bn, htri.data(), htri.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b + bn + bt, hinfo.data(), hinfo.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ctx->arena.free(blk);
    return device_fail(ctx, e, "mesh upload");
  }
  auto m = std::make_unique<DevMesh>();
  m->view.nodes = reinterpret_cast<const float4*>(b);
  m->view.tri = reinterpret_cast<const float4*>(b + bn);
  m->view.info = reinterpret_cast<const float*>(b + bn + bt);
  m->view.n_nodes = static_cast<int>(nn);
  m->view.n_faces = F;
  m->view.alpha = d->alpha;
  m->view.bulge = static_cast<float>(d->alpha * max_edge * (1.0 + 1e-6));
  m->block = blk;
  m->bytes = bn + bt + bi;
  m->volume = volume;
  m->max_edge = max_edge;
  const uint64_t id = ctx->next_id++;
  ctx->meshes[id] = std::move(m);
  *out = id;
  return GRASP_OK;
}

grasp_status grasp_unload_mesh(grasp_ctx* ctx, grasp_mesh_id id) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevMesh* m = find_mesh(ctx, id);
  if (!m) return fail(GRASP_EINVAL, "unknown mesh id");
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->arena.free(m->block);
  ctx->meshes.erase(id);
  return GRASP_OK;
}

grasp_status grasp_mesh_sample(grasp_ctx* ctx, grasp_mesh_id id, int32_t n, const float* r, float* out,
                               void* hip_stream) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (n < 0) return fail(GRASP_EINVAL, "n must be >= 0");
  if (n > 0 && (!r || !out)) return fail(GRASP_EINVAL, "r/out is NULL");
  MeshView v;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevMesh* m = find_mesh(ctx, id);
    if (!m) return fail(GRASP_EINVAL, "unknown mesh id");
    v = m->view;
  }
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_mesh_sample(v, n, r, out, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_mesh_sample launch");
  return GRASP_OK;
}

grasp_status grasp_debug_mesh_step_sample(grasp_ctx* ctx, grasp_mesh_id id, int32_t n, const float* r, float* out,
                                          void* hip_stream) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (n < 0) return fail(GRASP_EINVAL, "n must be >= 0");
  if (n > 0 && (!r || !out)) return fail(GRASP_EINVAL, "r/out is NULL");
  MeshView v;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevMesh* m = find_mesh(ctx, id);
    if (!m) return fail(GRASP_EINVAL, "unknown mesh id");
    v = m->view;
  }
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_mesh_step_sample(v, n, r, out, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_debug_mesh_step_sample launch");
  return GRASP_OK;
}

grasp_status grasp_load_sdf_from_mesh(grasp_ctx* ctx, grasp_mesh_id id, const grasp_mesh_grid_desc* d,
                                      grasp_sdf_id* out) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (!d || !out) return fail(GRASP_EINVAL, "desc/out is NULL");
  if (d->n < 2 || d->n > 512) return fail(GRASP_EINVAL, "n must be in [2, 512]");
  if (!(d->h > 0.0f) || !std::isfinite(d->h) || !std::isfinite(d->lo[0]) || !std::isfinite(d->lo[1]) ||
      !std::isfinite(d->lo[2]))
    return fail(GRASP_EINVAL, "h must be > 0 and lo finite");
  MeshView v;
  double volume;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevMesh* m = find_mesh(ctx, id);
    if (!m) return fail(GRASP_EINVAL, "unknown mesh id");
    v = m->view;
    volume = m->volume;
  }
  double Im = d->inertia_over_mass;
  if (!(Im > 0.0)) {
    const double Req = std::cbrt(3.0 * volume / (4.0 * M_PI));
    Im = 0.4 * Req * Req;
  }
  const int n = d->n;
  const float lo[3] = {d->lo[0], d->lo[1], d->lo[2]};
  const float h = d->h;
  return install_grid(ctx, n, d->lo, d->h, Im, d->layout,
                      [&](float* dev) { return launch_mesh_fill_grid(v, n, lo, h, dev, nullptr); }, out);
}

}  // extern "C"
