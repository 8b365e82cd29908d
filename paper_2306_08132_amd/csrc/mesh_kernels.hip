// The mesh object of Sec. III-B on gfx950: the Phong signed distance of a
// closed triangle mesh, queried through a bounding-volume hierarchy.
//
// One lane per query point (the grid fill: one wave per brick of grid
// vertices, walking together). The lane walks the hierarchy nearest child
// first with a private stack, pruning every box farther than the best
// triangle so far; the closest point of a triangle comes from its Voronoi
// regions (vertices, edges, interior). The sign is taken from the
// angle-weighted pseudonormal of the closest feature (face normal in the
// interior, the normalized sum of the two face normals on an edge, the
// angle-weighted vertex normal at a vertex), which for a closed mesh tells
// inside from outside exactly as a cast ray does. The Phong point moves the
// closest point r* towards the curved triangle,
//   p = r* - alpha sum_b w_b ((r* - v_b) . n_b) n_b,
// the same as (1 - alpha) r* + alpha sum_b w_b psi_b(r*) since the weights
// sum to one; rho = s |r - p| and grad rho = (r - p) / rho.
#include "device_common.h"
#include "internal.h"
#include "mesh_device.h"

namespace grasp {
namespace {

using namespace dev;
using namespace meshdev;

__global__ void k_mesh_sample(MeshView M, int n, const float* __restrict__ r, float* __restrict__ out4) {
  const int i = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float rho;
  V3 g;
  mesh_sdf(M, v3(r[3 * i], r[3 * i + 1], r[3 * i + 2]), rho, g);
  out4[4 * i] = rho;
  out4[4 * i + 1] = g.x;
  out4[4 * i + 2] = g.y;
  out4[4 * i + 3] = g.z;
}

// The sample the grasp step takes on a mesh: rho, the stated normal, the
// exact gradient of rho and the closest feature's region, [n][8].
__global__ void k_mesh_step_sample(MeshView M, int n, const float* __restrict__ r, float* __restrict__ out8) {
  const int i = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  MeshSample s;
  mesh_sample(M, v3(r[3 * i], r[3 * i + 1], r[3 * i + 2]), s);
  float* o = out8 + 8 * static_cast<size_t>(i);
  o[0] = s.rho;
  o[1] = s.n.x; o[2] = s.n.y; o[3] = s.n.z;
  o[4] = s.grad.x; o[5] = s.grad.y; o[6] = s.grad.z;
  o[7] = static_cast<float>(s.region);
}

// The grid's vertex (i, j, k) at lo + (i, j, k) h gets rho there. Each wave
// takes a 4 x 4 x 4 brick of vertices (lane = di + 4 dj + 16 dk), whose 64
// points walk the hierarchy together; lanes past the grid's edge only ride
// along.
__global__ void k_mesh_fill_grid(MeshView M, int n, float lox, float loy, float loz, float h,
                                 float* __restrict__ values) {
  const int nb = (n + 3) / 4;
  const long long brick = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (brick >= static_cast<long long>(nb) * nb * nb) return;  // whole waves
  const int lane = static_cast<int>(threadIdx.x) % kWave;
  const int i = 4 * static_cast<int>(brick % nb) + (lane & 3);
  const int j = 4 * static_cast<int>((brick / nb) % nb) + ((lane >> 2) & 3);
  const int k = 4 * static_cast<int>(brick / (static_cast<long long>(nb) * nb)) + (lane >> 4);
  const bool in = i < n && j < n && k < n;
  const V3 p = v3(fmaf(static_cast<float>(i), h, lox), fmaf(static_cast<float>(j), h, loy),
                  fmaf(static_cast<float>(k), h, loz));
  float best;
  const int f = nearest_triangle_wave(M, p, best, in);
  if (!in) return;
  float rho;
  V3 g;
  mesh_sdf_face(M, f, p, rho, g);
  values[(static_cast<long long>(k) * n + j) * n + i] = rho;
}

}  // namespace

hipError_t launch_mesh_sample(const MeshView& M, int n, const float* r, float* out4, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mesh_sample, dim3((n + 127) / 128), dim3(128), 0, stream, M, n, r, out4);
  return hipGetLastError();
}

hipError_t launch_mesh_step_sample(const MeshView& M, int n, const float* r, float* out8, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mesh_step_sample, dim3((n + 127) / 128), dim3(128), 0, stream, M, n, r, out8);
  return hipGetLastError();
}

hipError_t launch_mesh_fill_grid(const MeshView& M, int n, const float lo[3], float h, float* values,
                                 hipStream_t stream) {
  // one wave per 4^3 brick, two waves per workgroup
  const long long nb = (n + 3) / 4, waves = nb * nb * nb;
  hipLaunchKernelGGL(k_mesh_fill_grid, dim3(static_cast<unsigned>((waves + 1) / 2)), dim3(2 * kWave), 0, stream, M,
                     n, lo[0], lo[1], lo[2], h, values);
  return hipGetLastError();
}

}  // namespace grasp
