// Internal declarations shared by the host library and the gfx950 kernels of
// the grasp step. Not part of the public interface (see include/grasp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace grasp {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSims = 7;         // M velocity tests: +x, -x, +y, -y, +z, -z, 0
constexpr int kMaxLinks = 32;    // n_dof = 6 + (L - 1) <= 37 fits one wavefront
constexpr int kMaxDof = kMaxLinks + 5;
constexpr int kMaxDepth = 8;     // links on the path root -> leaf (root excluded)
constexpr int kLinkStride = 16;  // floats per link transform slot in LDS (3x4 + pad)

// A hand resident on the device. Contacts are re-laid out sorted by link, in
// structure-of-arrays form, padded to whole 64-contact chunks.
struct HandView {
  int L;            // links; link 0 = palm
  int n_dof;        // 6 + L - 1
  int Nc;           // contacts
  int n_chunks;     // ceil(Nc / 64)
  const float* origin;    // [L][12] row-major 3x4: parent frame -> joint, at q = 0
  const float* axis;      // [L][3] unit joint axis in the joint frame
  const int* parent;      // [L]; parent[0] = -1
  const int* chain;       // [L][kMaxDepth] links from the root's child down to l; -1 padded
  const int* depth;       // [L] number of valid chain entries
  const float* qlo;       // [n_dof]
  const float* qup;       // [n_dof]
  const float* cx;        // [n_chunks * 64] link-local contact coordinates, sorted by link and
  const float* cy;        //   within a link along a Morton curve of these coordinates
  const float* cz;
  const int* clink;       // [n_chunks * 64] link of each sorted contact (0 in padding)
  const int* chunk_lk;    // [n_chunks] first link | (last link << 16) of the chunk's valid contacts
  const int* link_start;  // [L + 1] first sorted contact of each link
  const int* perm;        // [Nc] sorted slot -> caller index
  const float* gcx;       // [n_chunks * 64] the same contacts in the Gauss-Seidel sweep order:
  const float* gcy;       //   sorted by link, the caller's order within a link (slot s has the
  const float* gcz;       //   same link in both orders)
};

// An object SDF resident on the device: vertex-centred N^3 grid, and the
// same values re-laid out with each cell's 8 corners contiguous (32 B).
struct SdfView {
  int n;
  float lo[3];
  float h;
  float inv_h;
  float inv_Im;            // 1 / (I/m)
  const float* values;     // [N^3], x fastest
  // Gather copy of the grid, one of two layouts:
  //  kLayoutYZQuads: [N-1][N-1][N] float4 per vertex, (phi(i,j,k), phi(i,j+1,k), phi(i,j,k+1), phi(i,j+1,k+1))
  //  kLayoutZPairs: [N-1][N][N] float2 per vertex, (phi(i,j,k), phi(i,j,k+1))
  const float4* cells;
  uint32_t cells_bytes;    // size of cells (< 4 GiB: buffer loads use 32-bit offsets)
  int layout;
  // Lower bounds for culling: for every block of kBlockCells^3 cells, the
  // minimum over the vertices of its cells widened by one cell on every side,
  // [nb][nb][nb] with nb = ceil((N-1) / kBlockCells).
  const float* bmin;
  int nb;
};

constexpr int kBlockShift = 2;
constexpr int kBlockCells = 1 << kBlockShift;

// Layouts of the gather copy. yz-quads hold a cell's 8 corners in 32
// contiguous bytes of one row, so a contact's seven test points, which lie in
// neighbouring cells, touch about four cache lines; z-pairs need two rows per
// sample but half the memory. yz-quads measured fastest from 96^3 to 256^3
// (at 96^3 the two tie) and are the default.
constexpr int kLayoutYZQuads = 0;
constexpr int kLayoutZPairs = 1;
// Not a grid layout: the step's object is a triangle mesh (MeshView), its
// Phong signed distance queried through the hierarchy at every sample.
constexpr int kLayoutMesh = 2;

// A triangle mesh resident on the device (Sec. III-B): a bounding-volume
// hierarchy in depth-first order and per-face records.
//  nodes: [n_nodes][2] float4 (lo.xyz, a), (hi.xyz, count): a leaf (count > 0)
//         holds faces [a, a + count); an internal node (count = 0) has its
//         children at node + 1 and a
//  tri:   [n_faces][3] float4 vertex positions (xyz), faces in leaf order
//  info:  [n_faces][kMeshInfo] floats: Phong normals of the three vertices,
//         face normal, pseudonormals of edges ab, bc, ca and of vertices a, b, c
struct MeshView {
  const float4* nodes;
  const float4* tri;
  const float* info;
  int n_nodes;
  int n_faces;
  float alpha;  // Phong blend
  float bulge;  // alpha times the longest edge (widened by 1e-6): the Phong point's largest offset
                // from the flat closest point, so rho >= (distance to the root box) - bulge
};

// Device copy of the step parameters.
struct StepConsts {
  float dt, v0, omega, r_dil, alpha, w_stable, w_pen, w_range, w_limit, w_min;
  float mu;     // Coulomb friction coefficient (0: frictionless; one iteration only)
  int K;        // projection iterations
  int ckpt;     // pose checkpoint interval (1 = every iteration kept)
};

struct AdamConsts {
  float lr, b1, b2, eps;
  float c1, c2;  // bias corrections 1 - b1^t, 1 - b2^t
};

// Per-wave LDS layout of the step kernel (floats): link transforms, joint
// frames, link wrench adjoints, per-test constants, a chunk's contact
// points, then pose checkpoints
// (K/ckpt + 1 slots) and a replay buffer (ckpt slots), each slot 7 x 6.
constexpr int kOffT = 0;                       // [kMaxLinks][12]
constexpr int kOffJ = kOffT + kMaxLinks * 12;  // [kMaxLinks][6] joint world origin, world axis
constexpr int kOffW = kOffJ + kMaxLinks * 6;   // [kMaxLinks][6] link force, torque adjoints
constexpr int kUStride = 32;
constexpr int kOffU = kOffW + kMaxLinks * 6;   // [7][32] per-test constants
constexpr int kOffWS = kOffU + kSims * kUStride;   // [7][6] summed corrections of the last pass,
                                                   // then [7] active-constraint counts (+7 pad)
constexpr int kOffCnt = kOffWS + kSims * 6;
constexpr int kOffP = kOffWS + 56;             // [64][4] world contact points of a chunk (x, y, z, link);
                                               // [6][64] per-lane sums at the end of a pass
constexpr int kOffPose = kOffP + kWave * 6;

// After the pose slots: the active-constraint count of every (iteration, test),
// [K][7], which sets the average of that iteration's corrections.
__host__ __device__ inline int pose_slots(int K, int ckpt) { return K / ckpt + 1; }
__host__ __device__ inline size_t counts_offset(int K, int ckpt) {
  return static_cast<size_t>(kOffPose) + static_cast<size_t>(K / ckpt + 1 + ckpt) * kSims * 6;
}
__host__ __device__ inline size_t wave_lds_floats(int K, int ckpt) {
  const size_t f = counts_offset(K, ckpt) + static_cast<size_t>(K) * kSims;
  return (f + 31) / 32 * 32;  // keep every wave's region 128-byte aligned
}

// What one launch of the step kernel does.
enum StepKind : int {
  STEP_FWD = 0,        // loss/terms; pose checkpoints to the workspace if given
  STEP_BWD = 1,        // dq from saved checkpoints (or recomputed forward)
  STEP_FUSED = 2,      // forward + backward (+ Adam) in one launch
};

struct StepArgs {
  HandView hand;
  SdfView sdf;
  StepConsts prm;
  AdamConsts adam;
  int B;
  const float* q;       // [B][n_dof]
  float* q_out;         // Adam: updated q (may alias q)
  float* m;             // Adam state [B][n_dof] (or null)
  float* v;
  float* loss;          // [B] (or null)
  float* terms;         // [B][4] (or null)
  float* dq;            // [B][n_dof] (or null)
  const float* dloss;   // [B] (or null: 1)
  float* poses;         // [B][slots][7][6] checkpoints, then [B][K][7] counts (or null)
  int* nonfinite;       // [1] set when any loss is not finite (or null)
  const int* order;     // [B] candidate taken by work item i (or null: i itself)
  unsigned long long* fwd_groups;  // [2] += (sample groups gathered, sample groups) over
                                   // every untraced forward pass (or null)
  // a mesh object (nodes set): the step samples its Phong signed distance
  // instead of the grid; sdf then carries only inv_Im
  MeshView mesh;
  int* mesh_face;       // [B][7][Nc] nearest face of every sample of a one-iteration mesh step,
                        // written by the forward and read by the adjoint (or null: both walk)
  // debug trace (caller order), all optional
  float* trace_p;       // [B][Nc][3]
  float* trace_poses;   // [B][7][K+1][6]
  float* trace_samples; // [B][7][K][Nc][6] = d, g, w, lambda
};

// Launch shape of the step kernel: waves (candidates) per workgroup and the
// minimum waves per SIMD its registers must allow. Every shape computes the
// same bits; only speed differs.
struct TileCfg {
  int wpb = 4;
  int occ = 1;
};
bool valid_tile(TileCfg c);

// The shape used where none was set or tuned. One iteration (128 VGPRs with
// 12 bytes of spills): two waves per workgroup at four per SIMD (16 uneven
// batched jobs 5.89 -> 5.52 ms against one wave per SIMD's minimum; the tuner
// picks it on the 4096-candidate step). Several iterations: one wave per
// workgroup at four per SIMD (128 VGPRs, 80 bytes of spills per lane; the
// 65536-candidate K = 16 step 568 -> 519 ms against two or three per SIMD at
// 152 VGPRs without spills; five per SIMD spill 252 bytes and take 1012 ms).
inline TileCfg default_tile(bool kone) { return kone ? TileCfg{2, 4} : TileCfg{1, 4}; }

hipError_t launch_step(const StepArgs& a, StepKind kind, bool adam, TileCfg cfg, hipStream_t stream);
// The same step on a mesh object (a.mesh): one projection form (averaged),
// no culling, two candidates per workgroup.
hipError_t launch_step_mesh(const StepArgs& a, StepKind kind, bool adam, hipStream_t stream);

// Candidates of at least this many get a locality order before the step.
constexpr int kOrderMinB = 256;
// Writes order[0..B) = a permutation of the candidates grouped by the
// direction of the wrist from the grid's centre (one workgroup).
hipError_t launch_order(const float* q, int n_dof, int B, const SdfView& S, int* order, hipStream_t stream);

// The plain per-job form (one projection iteration): workspace floats and
// the unfused stage kernels; *dq_out receives the workspace slot holding dq.
size_t plain_workspace_floats(const HandView& H, int B);
hipError_t launch_plain_step(const HandView& H, const SdfView& S, const StepConsts& P, int B, const float* q,
                             float* loss, float* terms, float* ws, float** dq_out, hipStream_t stream);

// Batched form: a device table of jobs, each one StepArgs for a fused step of
// its B candidates; items [begin, begin + B) of the shared work range.
struct BatchJob {
  StepArgs args;
  int begin;   // first item of the job in the table (sum of the earlier jobs' B)
  int slice;   // ceil(B / 8): the candidates of the job each XCD takes
  int begin8;  // sum of the earlier jobs' slices: the job's place in every XCD's list
  int pad;
};
struct BatchHeader {
  int n_jobs;
  int total;   // sum of B over the table
  int total8;  // sum of the slices
  int pad;
};
// Launches `blocks` workgroups (a multiple of 8) over the table; XCD x takes
// candidates [x slice, (x + 1) slice) of every job. Waves past the table exit;
// kone selects the one-iteration kernel (every job in the table must agree on it);
// fric, the several-iteration kernel with friction compiled in (needed when a job has mu > 0).
hipError_t launch_batch(const BatchHeader* hdr, const BatchJob* jobs, bool kone, bool fric, TileCfg cfg, int blocks,
                        int lds_floats, hipStream_t stream);

// The same for every job of a batch table whose order pointer is set.
hipError_t launch_order_batch(const BatchHeader* hdr, const BatchJob* jobs, int max_jobs, hipStream_t stream);

constexpr int kMeshInfo = 32;
constexpr int kMeshStack = 32;  // traversal stack entries; the hierarchy is kept shallower
hipError_t launch_mesh_sample(const MeshView& M, int n, const float* r, float* out4, hipStream_t stream);
hipError_t launch_mesh_step_sample(const MeshView& M, int n, const float* r, float* out8, hipStream_t stream);
hipError_t launch_mesh_fill_grid(const MeshView& M, int n, const float lo[3], float h, float* values,
                                 hipStream_t stream);

hipError_t launch_adam(int n, float* q, float* m, float* v, const float* g, AdamConsts c,
                       hipStream_t stream);
hipError_t launch_build_gather(const float* values, int n, int layout, float4* cells, hipStream_t stream);
hipError_t launch_build_bmin(const float* values, int n, float* bmin, hipStream_t stream);
hipError_t launch_sample_points(const SdfView& s, int n, const float* r, float* out4, float* hess9,
                                hipStream_t stream);

}  // namespace grasp
