// C-ABI entry points of the grasp-step library: context, arena, resident
// hands and SDF grids, and the step calls. Argument checking happens here so
// that kernels only ever see shapes they were written for.
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <numeric>
#include <string>
#include <vector>

#include "context.h"
#include "gs.h"

namespace grasp {

namespace {
thread_local std::string g_last_error;

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
bool finite(float x) { return std::isfinite(x); }
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

grasp_status fail(grasp_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
  ok_ = (prev_ == dev) || (hipSetDevice(dev) == hipSuccess);
}

DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
}

grasp_status device_fail(grasp_ctx* ctx, hipError_t e, const char* where) {
  if (ctx) ctx->poisoned = true;
  return fail(GRASP_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

DevHand* find_hand(grasp_ctx* ctx, grasp_hand_id id) {
  auto it = ctx->hands.find(id);
  return it == ctx->hands.end() ? nullptr : it->second.get();
}

DevSdf* find_sdf(grasp_ctx* ctx, grasp_sdf_id id) {
  auto it = ctx->sdfs.find(id);
  return it == ctx->sdfs.end() ? nullptr : it->second.get();
}

grasp_status check_params(const grasp_step_params* p, StepConsts* out) {
  if (!p) return fail(GRASP_EINVAL, "params is NULL");
  if (!(p->dt > 0.0f) || !finite(p->dt)) return fail(GRASP_EINVAL, "dt must be finite and > 0");
  if (!finite(p->v0)) return fail(GRASP_EINVAL, "v0 must be finite");
  if (p->K < 1 || p->K > 1024) return fail(GRASP_EINVAL, "K must be in [1, 1024]");
  if (p->ckpt_every < 1 || p->K % p->ckpt_every != 0)
    return fail(GRASP_EINVAL, "ckpt_every must be >= 1 and divide K");
  if (!finite(p->omega) || !finite(p->r_dil) || p->r_dil < 0.0f || !finite(p->alpha_leak) ||
      !finite(p->w_stable) || !finite(p->w_pen) || !finite(p->w_range) || !finite(p->w_limit) ||
      !finite(p->w_min) || p->w_min < 0.0f)
    return fail(GRASP_EINVAL, "params must be finite (r_dil, w_min >= 0)");
  if (p->mode < GRASP_MODE_AUTO || p->mode > GRASP_MODE_RECOMPUTE) return fail(GRASP_EINVAL, "bad mode");
  if (p->projection != GRASP_PROJECTION_AVERAGED && p->projection != GRASP_PROJECTION_GAUSS_SEIDEL)
    return fail(GRASP_EINVAL, "bad projection");
  if (!finite(p->mu) || p->mu < 0.0f) return fail(GRASP_EINVAL, "friction coefficient mu must be finite and >= 0");
  if (p->mu > 0.0f && p->projection != GRASP_PROJECTION_AVERAGED)
    return fail(GRASP_EINVAL, "friction (mu > 0) runs with the averaged projection");
  // LDS of one wave must fit comfortably: K/ckpt + 1 + ckpt pose slots
  if (wave_lds_floats(p->K, p->ckpt_every) * sizeof(float) > 16 * 1024)
    return fail(GRASP_EINVAL, "K / ckpt_every too large for the pose checkpoint buffer");
  if (out) {
    out->dt = p->dt;
    out->v0 = p->v0;
    out->omega = p->omega;
    out->r_dil = p->r_dil;
    out->alpha = p->alpha_leak;
    out->w_stable = p->w_stable;
    out->w_pen = p->w_pen;
    out->w_range = p->w_range;
    out->w_limit = p->w_limit;
    out->w_min = p->w_min;
    out->mu = p->mu;
    out->K = p->K;
    out->ckpt = p->ckpt_every;
  }
  return GRASP_OK;
}

}  // namespace grasp

using namespace grasp;

namespace {
void load_tile_cache(grasp_ctx* ctx);

// Candidate locality order of grasp_step_fused_static: a fixed device array
// (each GPU the library runs on holds its own copy until the process ends),
// so that step allocates nothing. Host code uses only the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
constexpr int kStaticOrderMax = 262144;  // candidates: 1 MiB of ints
static __device__ __align__(256) int scratch[kStaticOrderMax];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current: the device address of scratch.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<int*>(ptr);
  return hipSuccess;
}

int* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

#define GRASP_CHECK_CTX(ctx)                                                        \
  do {                                                                              \
    if (!(ctx)) return fail(GRASP_EINVAL, "context is NULL");                       \
    if ((ctx)->poisoned) return fail(GRASP_EDEVICE, "context poisoned by an earlier device error"); \
  } while (0)


}  // namespace

extern "C" {

const char* grasp_last_error(void) { return g_last_error.c_str(); }

grasp_status grasp_init(int device, void* arena_dev, size_t arena_bytes, grasp_ctx** out) {
  set_error("");
  if (!out) return fail(GRASP_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return fail(GRASP_EDEVICE, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
  if (device < 0 || device >= n) return fail(GRASP_EINVAL, "no such device");
  if (arena_bytes < kGranule) return fail(GRASP_EINVAL, "arena_bytes too small");
  if (arena_dev && (reinterpret_cast<uintptr_t>(arena_dev) % kGranule) != 0)
    return fail(GRASP_EINVAL, "arena must be 256-byte aligned");
  DeviceGuard g(device);
  if (!g.ok()) return fail(GRASP_EDEVICE, "hipSetDevice failed");
  auto* ctx = new grasp_ctx();
  ctx->device = device;
  if (arena_dev) {
    ctx->arena_base = static_cast<char*>(arena_dev);
  } else {
    void* p = nullptr;
    e = hipMalloc(&p, arena_bytes);
    if (e != hipSuccess) {
      delete ctx;
      return fail(GRASP_ENOMEM, std::string("hipMalloc arena: ") + hipGetErrorString(e));
    }
    ctx->arena_base = static_cast<char*>(p);
    ctx->arena_owned = true;
  }
  ctx->arena.reset(ctx->arena_base, arena_bytes);
  e = scratch_setup(device);
  if (e != hipSuccess) {
    if (ctx->arena_owned) (void)hipFree(ctx->arena_base);
    delete ctx;
    return fail(GRASP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  load_tile_cache(ctx);
  *out = ctx;
  return GRASP_OK;
}

void grasp_shutdown_scheduler(grasp_ctx* ctx);  // sched.cpp

void grasp_shutdown(grasp_ctx* ctx) {
  if (!ctx) return;
  grasp_shutdown_scheduler(ctx);
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->order_ev) (void)hipEventDestroy(ctx->order_ev);
    if (ctx->gs_ev) (void)hipEventDestroy(ctx->gs_ev);
    if (ctx->face_ev) (void)hipEventDestroy(ctx->face_ev);
    if (ctx->arena_owned) (void)hipFree(ctx->arena_base);
  }
  delete ctx;
}

void grasp_default_params(grasp_step_params* p) {
  if (!p) return;
  p->dt = 1e-3f;
  p->v0 = 1.0f;
  p->K = 1;
  p->ckpt_every = 1;
  p->omega = 1.0f;
  p->r_dil = 0.0f;
  p->alpha_leak = 0.1f;
  p->w_stable = 1.0f;
  p->w_pen = 1e4f;
  p->w_range = 1e-2f;
  p->w_limit = 1.0f;
  p->w_min = 1e-8f;
  p->mode = GRASP_MODE_AUTO;
  p->projection = GRASP_PROJECTION_AVERAGED;
  p->mu = 0.0f;
}

// ---------------------------------------------------------------------------
// hands
// ---------------------------------------------------------------------------
grasp_status grasp_create_hand(grasp_ctx* ctx, const grasp_hand_desc* d, grasp_hand_id* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!d || !out) return fail(GRASP_EINVAL, "desc/out is NULL");
  const int L = d->n_links, Nc = d->n_contacts;
  if (L < 1 || L > kMaxLinks) return fail(GRASP_EINVAL, "n_links must be in [1, 32]");
  if (Nc < 1 || Nc > (1 << 24)) return fail(GRASP_EINVAL, "n_contacts must be in [1, 2^24]");
  if (!d->parent || !d->joint_origin || !d->joint_axis || !d->q_low || !d->q_up || !d->contact_local ||
      !d->contact_link)
    return fail(GRASP_EINVAL, "hand description has a NULL array");
  const int nd = 6 + L - 1;
  if (d->parent[0] != -1) return fail(GRASP_EINVAL, "parent[0] must be -1");
  std::vector<int> depth(L, 0), chain(static_cast<size_t>(L) * kMaxDepth, -1);
  for (int l = 1; l < L; ++l) {
    if (d->parent[l] < 0 || d->parent[l] >= l) return fail(GRASP_EINVAL, "parent[l] must be in [0, l)");
    depth[l] = depth[d->parent[l]] + 1;
    if (depth[l] > kMaxDepth) return fail(GRASP_EINVAL, "chain deeper than 8 links");
    for (int s = 0; s < depth[l] - 1; ++s) chain[l * kMaxDepth + s] = chain[d->parent[l] * kMaxDepth + s];
    chain[l * kMaxDepth + depth[l] - 1] = l;
    const float* a = d->joint_axis + 3 * l;
    const float n = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (!(std::fabs(n - 1.0f) <= 1e-3f)) return fail(GRASP_EINVAL, "joint_axis must be unit length");
    for (int j = 0; j < 12; ++j)
      if (!finite(d->joint_origin[12 * l + j])) return fail(GRASP_EINVAL, "joint_origin not finite");
  }
  for (int j = 6; j < nd; ++j)
    if (!finite(d->q_low[j]) || !finite(d->q_up[j]) || d->q_low[j] > d->q_up[j])
      return fail(GRASP_EINVAL, "joint limits must be finite with q_low <= q_up");
  for (int i = 0; i < Nc; ++i) {
    if (d->contact_link[i] < 0 || d->contact_link[i] >= L) return fail(GRASP_EINVAL, "contact_link out of range");
    for (int j = 0; j < 3; ++j)
      if (!finite(d->contact_local[3 * i + j])) return fail(GRASP_EINVAL, "contact_local not finite");
  }
  // Two orders of the contacts, both sorted by link (so slot s has the same
  // link in both). The step's: within a link along a Morton curve of the
  // link-frame coordinates (10 bits per axis over the link's box), so that
  // the contacts sharing a wave instruction, and the next ones, sample
  // neighbouring grid cells. The Gauss-Seidel sweep's: the caller's order
  // within a link (the sweep order is part of that projection's result).
  // Each maps slot -> caller index.
  std::vector<float> blo(3 * static_cast<size_t>(L), INFINITY), bhi(3 * static_cast<size_t>(L), -INFINITY);
  for (int i = 0; i < Nc; ++i)
    for (int j = 0; j < 3; ++j) {
      const int l = d->contact_link[i];
      blo[3 * l + j] = std::min(blo[3 * l + j], d->contact_local[3 * i + j]);
      bhi[3 * l + j] = std::max(bhi[3 * l + j], d->contact_local[3 * i + j]);
    }
  auto spread = [](uint64_t v) {  // 10 bits -> every third bit
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x30000ff;
    v = (v | (v << 8)) & 0x300f00f;
    v = (v | (v << 4)) & 0x30c30c3;
    v = (v | (v << 2)) & 0x9249249;
    return v;
  };
  std::vector<uint64_t> key(Nc);
  for (int i = 0; i < Nc; ++i) {
    const int l = d->contact_link[i];
    uint64_t m = 0;
    for (int j = 0; j < 3; ++j) {
      const float ext = bhi[3 * l + j] - blo[3 * l + j];
      const float u = ext > 0.0f ? (d->contact_local[3 * i + j] - blo[3 * l + j]) / ext : 0.0f;
      m |= spread(static_cast<uint64_t>(std::min(1023.0f, std::max(0.0f, u * 1023.0f)))) << j;
    }
    key[i] = (static_cast<uint64_t>(l) << 32) | m;
  }
  std::vector<int> perm(Nc);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<int> gperm(Nc);
  std::iota(gperm.begin(), gperm.end(), 0);
  std::stable_sort(gperm.begin(), gperm.end(), [&](int a, int b) { return d->contact_link[a] < d->contact_link[b]; });
  const int nch = (Nc + kWave - 1) / kWave;
  const int npad = nch * kWave;
  std::vector<float> cx(npad, 0.0f), cy(npad, 0.0f), cz(npad, 0.0f), gx(npad, 0.0f), gy(npad, 0.0f), gz(npad, 0.0f);
  std::vector<int> clink(npad, 0), chunk(nch, 0), link_start(L + 1, 0);
  for (int s = 0; s < Nc; ++s) {
    const int i = perm[s], k = gperm[s];
    cx[s] = d->contact_local[3 * i];
    cy[s] = d->contact_local[3 * i + 1];
    cz[s] = d->contact_local[3 * i + 2];
    gx[s] = d->contact_local[3 * k];
    gy[s] = d->contact_local[3 * k + 1];
    gz[s] = d->contact_local[3 * k + 2];
    clink[s] = d->contact_link[i];
  }
  for (int s = 0; s < Nc; ++s) link_start[clink[s] + 1] = s + 1;
  for (int l = 1; l <= L; ++l) link_start[l] = std::max(link_start[l], link_start[l - 1]);
  for (int c = 0; c < nch; ++c) {
    const int first = clink[c * kWave];
    const int last = clink[std::min(Nc, (c + 1) * kWave) - 1];
    chunk[c] = first | (last << 16);
  }
  std::vector<float> origin(static_cast<size_t>(L) * 12), axis(static_cast<size_t>(L) * 3), qlo(nd), qup(nd);
  std::memcpy(origin.data(), d->joint_origin, origin.size() * sizeof(float));
  std::memcpy(axis.data(), d->joint_axis, axis.size() * sizeof(float));
  std::memcpy(qlo.data(), d->q_low, nd * sizeof(float));
  std::memcpy(qup.data(), d->q_up, nd * sizeof(float));
  for (int j = 0; j < 6; ++j) { qlo[j] = 0.0f; qup[j] = 0.0f; }
  std::vector<int> parent(d->parent, d->parent + L);

  // one device block: floats, then ints
  struct Part { const void* src; size_t bytes; size_t off; };
  std::vector<Part> parts = {
      {origin.data(), origin.size() * 4, 0}, {axis.data(), axis.size() * 4, 0}, {qlo.data(), qlo.size() * 4, 0},
      {qup.data(), qup.size() * 4, 0},       {cx.data(), cx.size() * 4, 0},     {cy.data(), cy.size() * 4, 0},
      {cz.data(), cz.size() * 4, 0},         {parent.data(), parent.size() * 4, 0},
      {chain.data(), chain.size() * 4, 0},   {depth.data(), depth.size() * 4, 0},
      {clink.data(), clink.size() * 4, 0},   {chunk.data(), chunk.size() * 4, 0},
      {perm.data(), perm.size() * 4, 0},     {link_start.data(), link_start.size() * 4, 0},
      {gx.data(), gx.size() * 4, 0},         {gy.data(), gy.size() * 4, 0},
      {gz.data(), gz.size() * 4, 0}};
  size_t total = 0;
  for (auto& p : parts) { p.off = total; total += round_up(p.bytes, 256); }
  std::vector<char> host(total, 0);
  for (auto& p : parts) std::memcpy(host.data() + p.off, p.src, p.bytes);

  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(GRASP_EDEVICE, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(ctx->mu);
  void* blk = ctx->arena.alloc(total);
  if (!blk) return fail(GRASP_ENOMEM, "arena full (hand)");
  hipError_t e = hipMemcpy(blk, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ctx->arena.free(blk);
    return device_fail(ctx, e, "hipMemcpy hand");
  }
  auto h = std::make_unique<DevHand>();
  char* b = static_cast<char*>(blk);
  auto F = [&](int k) { return reinterpret_cast<const float*>(b + parts[k].off); };
  auto I = [&](int k) { return reinterpret_cast<const int*>(b + parts[k].off); };
  h->view.L = L;
  h->view.n_dof = nd;
  h->view.Nc = Nc;
  h->view.n_chunks = nch;
  h->view.origin = F(0);
  h->view.axis = F(1);
  h->view.qlo = F(2);
  h->view.qup = F(3);
  h->view.cx = F(4);
  h->view.cy = F(5);
  h->view.cz = F(6);
  h->view.parent = I(7);
  h->view.chain = I(8);
  h->view.depth = I(9);
  h->view.clink = I(10);
  h->view.chunk_lk = I(11);
  h->view.perm = I(12);
  h->view.link_start = I(13);
  h->view.gcx = F(14);
  h->view.gcy = F(15);
  h->view.gcz = F(16);
  h->block = blk;
  h->bytes = total;
  h->contact_link.assign(d->contact_link, d->contact_link + Nc);
  const uint64_t id = ctx->next_id++;
  ctx->hands[id] = std::move(h);
  *out = id;
  return GRASP_OK;
}

grasp_status grasp_destroy_hand(grasp_ctx* ctx, grasp_hand_id id) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevHand* h = find_hand(ctx, id);
  if (!h) return fail(GRASP_EINVAL, "unknown hand id");
  if (h->live_jobs > 0) return fail(GRASP_EBUSY, "hand in use by a live job");
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->arena.free(h->block);
  ctx->hands.erase(id);
  return GRASP_OK;
}

grasp_status grasp_hand_contact_links(grasp_ctx* ctx, grasp_hand_id id, int32_t* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!out) return fail(GRASP_EINVAL, "out is NULL");
  HandView v;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevHand* h = find_hand(ctx, id);
    if (!h) return fail(GRASP_EINVAL, "unknown hand id");
    v = h->view;
  }
  DeviceGuard g(ctx->device);
  std::vector<int> clink(v.Nc), perm(v.Nc);
  hipError_t e = hipMemcpy(clink.data(), v.clink, v.Nc * sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(perm.data(), v.perm, v.Nc * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(ctx, e, "hipMemcpy contact links");
  for (int s = 0; s < v.Nc; ++s) {
    if (perm[s] < 0 || perm[s] >= v.Nc) return fail(GRASP_EINVAL, "corrupt contact permutation");
    out[perm[s]] = clink[s];
  }
  return GRASP_OK;
}

}  // extern "C"

namespace grasp {

grasp_status install_grid(grasp_ctx* ctx, int n_, const float lo[3], float h, double Im, int layout_req,
                          const std::function<hipError_t(float*)>& fill, grasp_sdf_id* out) {
  const size_t n = static_cast<size_t>(n_);
  const size_t n3 = n * n * n;
  const size_t nc = n - 1;
  const size_t vbytes = round_up(n3 * sizeof(float), 256);
  if (layout_req < GRASP_LAYOUT_AUTO || layout_req > GRASP_LAYOUT_ZPAIRS) return fail(GRASP_EINVAL, "unknown layout");
  const int layout = layout_req == GRASP_LAYOUT_ZPAIRS ? kLayoutZPairs : kLayoutYZQuads;
  // z-pairs: [n-1][n][n] x 8 bytes; yz-quads: [n-1][n-1][n] x 16 bytes
  const size_t cbytes = layout == kLayoutZPairs ? n * n * nc * 2 * sizeof(float) : n * nc * nc * 4 * sizeof(float);
  const int nb = static_cast<int>((nc + kBlockCells - 1) / kBlockCells);
  const size_t bbytes = round_up(static_cast<size_t>(nb) * nb * nb * sizeof(float), 256);
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(GRASP_EDEVICE, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(ctx->mu);
  void* blk = ctx->arena.alloc(vbytes + bbytes + cbytes);
  if (!blk) return fail(GRASP_ENOMEM, "arena full (SDF grid)");
  char* b = static_cast<char*>(blk);
  hipError_t e = fill(reinterpret_cast<float*>(b));
  if (e == hipSuccess)
    e = launch_build_gather(reinterpret_cast<const float*>(b), n_, layout,
                            reinterpret_cast<float4*>(b + vbytes + bbytes), nullptr);
  if (e == hipSuccess)
    e = launch_build_bmin(reinterpret_cast<const float*>(b), n_, reinterpret_cast<float*>(b + vbytes), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    ctx->arena.free(blk);
    return device_fail(ctx, e, "SDF upload");
  }
  auto s = std::make_unique<DevSdf>();
  s->view.n = n_;
  s->view.lo[0] = lo[0];
  s->view.lo[1] = lo[1];
  s->view.lo[2] = lo[2];
  s->view.h = h;
  s->view.inv_h = 1.0f / h;
  s->view.inv_Im = static_cast<float>(1.0 / Im);
  s->view.values = reinterpret_cast<const float*>(b);
  s->view.cells = reinterpret_cast<const float4*>(b + vbytes + bbytes);
  s->view.cells_bytes = static_cast<uint32_t>(cbytes);
  s->view.layout = layout;
  s->view.bmin = reinterpret_cast<const float*>(b + vbytes);
  s->view.nb = nb;
  s->block = blk;
  s->bytes = vbytes + bbytes + cbytes;
  s->inertia_over_mass = static_cast<float>(Im);
  const uint64_t id = ctx->next_id++;
  ctx->sdfs[id] = std::move(s);
  *out = id;
  return GRASP_OK;
}

}  // namespace grasp

extern "C" {

// ---------------------------------------------------------------------------
// SDF grids
// ---------------------------------------------------------------------------
grasp_status grasp_load_sdf(grasp_ctx* ctx, const grasp_sdf_desc* d, grasp_sdf_id* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!d || !out || !d->values) return fail(GRASP_EINVAL, "desc/out/values is NULL");
  if (d->n < 2 || d->n > 512) return fail(GRASP_EINVAL, "n must be in [2, 512]");
  if (!(d->h > 0.0f) || !finite(d->h) || !finite(d->lo[0]) || !finite(d->lo[1]) || !finite(d->lo[2]))
    return fail(GRASP_EINVAL, "h must be > 0 and lo finite");
  const size_t n = static_cast<size_t>(d->n);
  const size_t n3 = n * n * n;
  size_t neg = 0;
  for (size_t i = 0; i < n3; ++i) {
    if (!finite(d->values[i])) return fail(GRASP_EINVAL, "SDF values must be finite");
    neg += d->values[i] < 0.0f;
  }
  double Im = d->inertia_over_mass;
  if (!(Im > 0.0)) {
    // isotropic inertia of a uniform ball of the object's volume
    const double hh = d->h;
    const double V = hh * hh * hh * static_cast<double>(neg);
    if (neg == 0) return fail(GRASP_EINVAL, "object has no interior vertex; give inertia_over_mass");
    const double Req = std::cbrt(3.0 * V / (4.0 * M_PI));
    Im = 0.4 * Req * Req;
  }
  const float* host = d->values;
  return install_grid(ctx, d->n, d->lo, d->h, Im, d->layout,
                      [&](float* dev) { return hipMemcpy(dev, host, n3 * sizeof(float), hipMemcpyHostToDevice); },
                      out);
}

grasp_status grasp_unload_sdf(grasp_ctx* ctx, grasp_sdf_id id) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevSdf* s = find_sdf(ctx, id);
  if (!s) return fail(GRASP_EINVAL, "unknown sdf id");
  if (s->live_jobs > 0) return fail(GRASP_EBUSY, "SDF in use by a live job");
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->arena.free(s->block);
  ctx->sdfs.erase(id);
  return GRASP_OK;
}

grasp_status grasp_sdf_inertia(grasp_ctx* ctx, grasp_sdf_id id, float* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!out) return fail(GRASP_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevSdf* s = find_sdf(ctx, id);
  if (!s) return fail(GRASP_EINVAL, "unknown sdf id");
  *out = s->inertia_over_mass;
  return GRASP_OK;
}

// ---------------------------------------------------------------------------
// steps
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct Resolved {
  HandView hand;
  SdfView sdf;
  StepConsts prm;
};

// gs_ok: the entry point also runs the Gauss-Seidel projection (single-job
// fwd, bwd and fused steps).
grasp_status resolve(grasp_ctx* ctx, grasp_hand_id hid, grasp_sdf_id sid, const grasp_step_params* p, int32_t B,
                     Resolved* r, bool gs_ok = false) {
  if (B < 0) return fail(GRASP_EINVAL, "B must be >= 0");
  grasp_status st = check_params(p, &r->prm);
  if (st != GRASP_OK) return st;
  if (p->projection == GRASP_PROJECTION_GAUSS_SEIDEL) {
    if (!gs_ok)
      return fail(GRASP_EINVAL, "Gauss-Seidel projection runs in grasp_step_fwd, grasp_step_bwd and grasp_step_fused");
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevHand* h = find_hand(ctx, hid);
  if (!h) return fail(GRASP_EINVAL, "unknown hand id");
  DevSdf* s = find_sdf(ctx, sid);
  if (!s) return fail(GRASP_EINVAL, "unknown sdf id");
  r->hand = h->view;
  r->sdf = s->view;
  return GRASP_OK;
}

// Problem shape that a tuned tile belongs to: iteration structure, hand and
// grid sizes, and the candidate count rounded to a power of two.
std::string shape_key(const Resolved& r, int32_t B) {
  int bb = 1;
  while (bb < B) bb <<= 1;
  std::ostringstream os;
  os << "K" << r.prm.K << "c" << r.prm.ckpt << "L" << r.hand.L << "N" << r.hand.Nc << "g" << r.sdf.n << "B" << bb;
  return os.str();
}

TileCfg tile_for(grasp_ctx* ctx, const Resolved& r, int32_t B) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->tiles.find(shape_key(r, B));
  return it == ctx->tiles.end() ? default_tile(r.prm.K == 1) : it->second;
}

void load_tile_cache(grasp_ctx* ctx) {
  const char* path = std::getenv("GRASP_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string key;
  TileCfg c;
  while (f >> key >> c.wpb >> c.occ)
    if (valid_tile(c)) ctx->tiles[key] = c;
}

void save_tile(const std::string& key, TileCfg c) {
  const char* path = std::getenv("GRASP_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << c.wpb << " " << c.occ << "\n";
}

size_t pose_ws_bytes(const StepConsts& c, int32_t B) {
  // pose checkpoints [B][slots][7][6], then active-constraint counts [B][K][7]
  return static_cast<size_t>(B) * kSims * (pose_slots(c.K, c.ckpt) * 6 + c.K) * sizeof(float);
}

StepArgs base_args(const Resolved& r, int32_t B) {
  StepArgs a{};
  a.hand = r.hand;
  a.sdf = r.sdf;
  a.prm = r.prm;
  a.B = B;
  return a;
}

AdamConsts adam_consts(int32_t t, float lr, float b1, float b2, float eps) {
  AdamConsts c;
  c.lr = lr;
  c.b1 = b1;
  c.b2 = b2;
  c.eps = eps;
  c.c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), t));
  c.c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), t));
  return c;
}

grasp_status check_adam(int32_t t, float lr, float b1, float b2, float eps) {
  if (t < 1) return fail(GRASP_EINVAL, "Adam step t must be >= 1");
  if (!std::isfinite(lr) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps >= 0.0f) ||
      !std::isfinite(eps))
    return fail(GRASP_EINVAL, "bad Adam hyper-parameters");
  return GRASP_OK;
}

// The Gauss-Seidel step. A launch with a backward records where every chunk's
// sweep starts, in an arena buffer of the context shared by every stream:
// each use waits (on the device) for the previous one.
grasp_status launch_gs(grasp_ctx* ctx, const StepArgs& a, StepKind kind, bool adam, hipStream_t s,
                       const char* where) {
  if (a.B <= 0) return GRASP_OK;
  hipError_t e = hipSuccess;
  if (kind == STEP_FWD) {
    e = launch_gs_step(a, kind, adam, nullptr, s);
    return e == hipSuccess ? GRASP_OK : device_fail(ctx, e, where);
  }
  // the start-pose table is a context buffer that a later, larger step may
  // move: a captured graph would keep its old address
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return device_fail(ctx, e, where);
  if (cap != hipStreamCaptureStatusNone)
    return fail(GRASP_EINVAL, "a Gauss-Seidel step with a backward cannot be captured into a graph");
  const size_t need = gs_scratch_floats(a.B, a.hand.n_chunks, a.prm.K);
  std::lock_guard<std::mutex> lk(ctx->gs_mu);
  if (ctx->gs_cap < need) {
    // the old buffer may still be read by a launch on another stream
    if (ctx->gs_ev) e = hipEventSynchronize(ctx->gs_ev);
    if (e != hipSuccess) return device_fail(ctx, e, where);
    std::lock_guard<std::mutex> lka(ctx->mu);
    if (ctx->gs_buf) ctx->arena.free(ctx->gs_buf);
    ctx->gs_buf = static_cast<float*>(ctx->arena.alloc(need * sizeof(float)));
    ctx->gs_cap = ctx->gs_buf ? need : 0;
    if (!ctx->gs_buf) return fail(GRASP_ENOMEM, "arena full (Gauss-Seidel start poses)");
  }
  if (!ctx->gs_ev) e = hipEventCreateWithFlags(&ctx->gs_ev, hipEventDisableTiming);
  else e = hipStreamWaitEvent(s, ctx->gs_ev, 0);
  if (e == hipSuccess) e = launch_gs_step(a, kind, adam, ctx->gs_buf, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->gs_ev, s);
  return e == hipSuccess ? GRASP_OK : device_fail(ctx, e, where);
}

}  // namespace

// Runs launch(order) with the candidates of q in locality order (order =
// null when there are too few, the stream is being captured or the arena
// has no room): one arena buffer of the context shared by every stream,
// each use waiting (on the device) for the previous one.
hipError_t grasp::launch_with_order(grasp_ctx* ctx, const float* q, int n_dof, int B, const SdfView& S,
                                    hipStream_t s, const std::function<hipError_t(const int*)>& launch) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return e;
  if (B < kOrderMinB || cap != hipStreamCaptureStatusNone) return launch(nullptr);
  std::lock_guard<std::mutex> lk(ctx->order_mu);
  if (ctx->order_cap < B) {
    // the old buffer may still be read by a launch on another stream
    if (ctx->order_ev) e = hipEventSynchronize(ctx->order_ev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lka(ctx->mu);
    if (ctx->order_buf) ctx->arena.free(ctx->order_buf);
    ctx->order_buf = static_cast<int*>(ctx->arena.alloc(static_cast<size_t>(B) * sizeof(int)));
    ctx->order_cap = ctx->order_buf ? B : 0;
  }
  if (!ctx->order_buf) return launch(nullptr);
  if (!ctx->order_ev) e = hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming);
  else e = hipStreamWaitEvent(s, ctx->order_ev, 0);
  if (e == hipSuccess) e = launch_order(q, n_dof, B, S, ctx->order_buf, s);
  if (e == hipSuccess) e = launch(ctx->order_buf);
  if (e == hipSuccess) e = hipEventRecord(ctx->order_ev, s);
  return e;
}

namespace {

// One single-job step launch with the candidate locality order (B >= kOrderMinB,
// not under stream capture): the order kernel and the step run on stream s
// after the previous user of the context's order buffer, on any stream, has
// finished with it. Without memory for the buffer the step runs unordered.
hipError_t launch_ordered_step(grasp_ctx* ctx, StepArgs a, StepKind kind, bool adam, TileCfg tc, hipStream_t s) {
  return launch_with_order(ctx, a.q, a.hand.n_dof, a.B, a.sdf, s, [&](const int* order) {
    a.order = order;
    return launch_step(a, kind, adam, tc, s);
  });
}

}  // namespace

extern "C" {

grasp_status grasp_step_workspace_bytes(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                        const grasp_step_params* p, int32_t B, size_t* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!out) return fail(GRASP_EINVAL, "out is NULL");
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, true);
  if (st != GRASP_OK) return st;
  *out = p->projection == GRASP_PROJECTION_GAUSS_SEIDEL ? 0 : pose_ws_bytes(r.prm, B);
  return GRASP_OK;
}

grasp_status grasp_step_fwd(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                            int32_t B, const float* q, float* loss, float* terms, void* ws, size_t ws_bytes,
                            void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, true);
  if (st != GRASP_OK) return st;
  if (B > 0 && (!q || !loss)) return fail(GRASP_EINVAL, "q/loss is NULL");
  if (p->projection == GRASP_PROJECTION_GAUSS_SEIDEL) {
    StepArgs a = base_args(r, B);
    a.q = q;
    a.loss = loss;
    a.terms = terms;
    DeviceGuard g(ctx->device);
    return launch_gs(ctx, a, STEP_FWD, false, static_cast<hipStream_t>(hip_stream), "grasp_step_fwd launch");
  }
  const bool save = p->mode == GRASP_MODE_SAVE || (p->mode == GRASP_MODE_AUTO && ws);
  if (save && (!ws || ws_bytes < pose_ws_bytes(r.prm, B)))
    return fail(GRASP_ENOMEM, "workspace too small for SAVE mode");
  StepArgs a = base_args(r, B);
  a.q = q;
  a.loss = loss;
  a.terms = terms;
  a.poses = save ? static_cast<float*>(ws) : nullptr;
  const TileCfg tc = tile_for(ctx, r, B);
  DeviceGuard g(ctx->device);
  hipError_t e = launch_ordered_step(ctx, a, STEP_FWD, false, tc, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fwd launch");
  return GRASP_OK;
}

grasp_status grasp_step_bwd(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                            int32_t B, const float* q, const float* dloss, float* dq, void* ws, size_t ws_bytes,
                            void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, true);
  if (st != GRASP_OK) return st;
  if (B > 0 && (!q || !dq)) return fail(GRASP_EINVAL, "q/dq is NULL");
  if (p->projection == GRASP_PROJECTION_GAUSS_SEIDEL) {
    StepArgs a = base_args(r, B);
    a.q = q;
    a.dloss = dloss;
    a.dq = dq;
    DeviceGuard g(ctx->device);
    return launch_gs(ctx, a, STEP_BWD, false, static_cast<hipStream_t>(hip_stream), "grasp_step_bwd launch");
  }
  const bool save = p->mode == GRASP_MODE_SAVE || (p->mode == GRASP_MODE_AUTO && ws);
  if (save && (!ws || ws_bytes < pose_ws_bytes(r.prm, B)))
    return fail(GRASP_ENOMEM, "workspace too small for SAVE mode");
  StepArgs a = base_args(r, B);
  a.q = q;
  a.dloss = dloss;
  a.dq = dq;
  a.poses = save ? static_cast<float*>(ws) : nullptr;
  const TileCfg tc = tile_for(ctx, r, B);
  DeviceGuard g(ctx->device);
  hipError_t e = launch_ordered_step(ctx, a, STEP_BWD, false, tc, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_bwd launch");
  return GRASP_OK;
}

grasp_status grasp_adam_step(grasp_ctx* ctx, int32_t n, float* q, float* m, float* v, const float* g, int32_t t,
                             float lr, float b1, float b2, float eps, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (n < 0) return fail(GRASP_EINVAL, "n must be >= 0");
  if (n > 0 && (!q || !m || !v || !g)) return fail(GRASP_EINVAL, "q/m/v/g is NULL");
  grasp_status st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  DeviceGuard gd(ctx->device);
  hipError_t e = launch_adam(n, q, m, v, g, adam_consts(t, lr, b1, b2, eps), static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_adam_step launch");
  return GRASP_OK;
}

grasp_status grasp_step_fused(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                              int32_t B, float* q, float* m, float* v, int32_t t, float lr, float b1, float b2,
                              float eps, float* loss, float* terms, float* dq, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, true);
  if (st != GRASP_OK) return st;
  if (B > 0 && (!q || !m || !v)) return fail(GRASP_EINVAL, "q/m/v is NULL");
  st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  StepArgs a = base_args(r, B);
  a.q = q;
  a.q_out = q;
  a.m = m;
  a.v = v;
  a.loss = loss;
  a.terms = terms;
  a.dq = dq;
  a.adam = adam_consts(t, lr, b1, b2, eps);
  DeviceGuard g(ctx->device);
  if (p->projection == GRASP_PROJECTION_GAUSS_SEIDEL)
    return launch_gs(ctx, a, STEP_FUSED, true, static_cast<hipStream_t>(hip_stream), "grasp_step_fused launch");
  const TileCfg tc = tile_for(ctx, r, B);
  hipError_t e = launch_ordered_step(ctx, a, STEP_FUSED, true, tc, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused launch");
  return GRASP_OK;
}

namespace {
// The hand and the mesh of a mesh step, the parameters checked, and the I/m
// (<= 0: from the mesh's volume) into a.sdf.inv_Im.
grasp_status resolve_mesh(grasp_ctx* ctx, grasp_hand_id hand, grasp_mesh_id mesh, const grasp_step_params* p,
                          float inertia_over_mass, int32_t B, StepArgs* a) {
  if (B < 0) return fail(GRASP_EINVAL, "B must be >= 0");
  StepConsts prm;
  grasp_status st = check_params(p, &prm);
  if (st != GRASP_OK) return st;
  if (p->projection != GRASP_PROJECTION_AVERAGED)
    return fail(GRASP_EINVAL, "the step on a mesh runs the averaged projection only");
  if (p->mu != 0.0f) return fail(GRASP_EINVAL, "the step on a mesh is frictionless (mu = 0)");
  if (std::isnan(inertia_over_mass) || std::isinf(inertia_over_mass))
    return fail(GRASP_EINVAL, "inertia_over_mass must be finite");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DevHand* h = find_hand(ctx, hand);
  if (!h) return fail(GRASP_EINVAL, "unknown hand id");
  auto it = ctx->meshes.find(mesh);
  if (it == ctx->meshes.end()) return fail(GRASP_EINVAL, "unknown mesh id");
  a->hand = h->view;
  a->mesh = it->second->view;
  double Im = inertia_over_mass;
  if (!(Im > 0.0)) {
    const double Req = std::cbrt(3.0 * it->second->volume / (4.0 * M_PI));
    Im = 0.4 * Req * Req;
  }
  a->sdf.inv_Im = static_cast<float>(1.0 / static_cast<double>(static_cast<float>(Im)));
  a->prm = prm;
  a->B = B;
  return GRASP_OK;
}
}  // namespace

grasp_status grasp_debug_trace_mesh(grasp_ctx* ctx, grasp_hand_id hand, grasp_mesh_id mesh,
                                    const grasp_step_params* p, float inertia_over_mass, int32_t B, const float* q,
                                    float* p_world, float* poses, float* samples, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  StepArgs a{};
  grasp_status st = resolve_mesh(ctx, hand, mesh, p, inertia_over_mass, B, &a);
  if (st != GRASP_OK) return st;
  if (B > 0 && !q) return fail(GRASP_EINVAL, "q is NULL");
  a.q = q;
  a.trace_p = p_world;
  a.trace_poses = poses;
  a.trace_samples = samples;
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_step_mesh(a, STEP_FWD, false, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_debug_trace_mesh launch");
  return GRASP_OK;
}

grasp_status grasp_step_fused_mesh(grasp_ctx* ctx, grasp_hand_id hand, grasp_mesh_id mesh,
                                   const grasp_step_params* p, float inertia_over_mass, int32_t B, float* q, float* m,
                                   float* v, int32_t t, float lr, float b1, float b2, float eps, float* loss,
                                   float* terms, float* dq, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  StepArgs a{};
  grasp_status st = resolve_mesh(ctx, hand, mesh, p, inertia_over_mass, B, &a);
  if (st != GRASP_OK) return st;
  if (B > 0 && (!q || !m || !v)) return fail(GRASP_EINVAL, "q/m/v is NULL");
  st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  a.q = q;
  a.q_out = q;
  a.m = m;
  a.v = v;
  a.loss = loss;
  a.terms = terms;
  a.dq = dq;
  a.adam = adam_consts(t, lr, b1, b2, eps);
  DeviceGuard g(ctx->device);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (a.prm.K == 1 && B > 0) {
    // One iteration: the forward records each sample's nearest face in a
    // context buffer and the adjoint reuses it instead of walking the
    // hierarchy again. Not under stream capture (a later, larger step may
    // move the buffer) and not without room in the arena: then both walk.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused_mesh");
    if (cap == hipStreamCaptureStatusNone) {
      const size_t need = static_cast<size_t>(B) * kSims * static_cast<size_t>(a.hand.Nc);
      std::lock_guard<std::mutex> lk(ctx->face_mu);
      if (ctx->face_cap < need) {
        // the old buffer may still be in use by a launch on another stream
        if (ctx->face_ev) e = hipEventSynchronize(ctx->face_ev);
        if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused_mesh");
        std::lock_guard<std::mutex> lka(ctx->mu);
        if (ctx->face_buf) ctx->arena.free(ctx->face_buf);
        ctx->face_buf = static_cast<int*>(ctx->arena.alloc(need * sizeof(int)));
        ctx->face_cap = ctx->face_buf ? need : 0;
      }
      if (ctx->face_buf) {
        if (!ctx->face_ev) e = hipEventCreateWithFlags(&ctx->face_ev, hipEventDisableTiming);
        else e = hipStreamWaitEvent(s, ctx->face_ev, 0);
        a.mesh_face = ctx->face_buf;
        if (e == hipSuccess) e = launch_step_mesh(a, STEP_FUSED, true, s);
        if (e == hipSuccess) e = hipEventRecord(ctx->face_ev, s);
        if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused_mesh launch");
        return GRASP_OK;
      }
    }
  }
  e = launch_step_mesh(a, STEP_FUSED, true, s);
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused_mesh launch");
  return GRASP_OK;
}

grasp_status grasp_step_fused_static(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                     const grasp_step_params* p, int32_t B, float* q, float* m, float* v, int32_t t,
                                     float lr, float b1, float b2, float eps, float* loss, float* terms, float* dq,
                                     void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, false);
  if (st != GRASP_OK) return st;
  if (B > kStaticOrderMax)
    return fail(GRASP_EINVAL, "B exceeds the 262144 candidates of the static scratch (use grasp_step_fused)");
  if (B > 0 && (!q || !m || !v)) return fail(GRASP_EINVAL, "q/m/v is NULL");
  st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  int* order = scratch_of(ctx->device);
  if (!order) return fail(GRASP_EDEVICE, "static scratch not set up for this device");
  StepArgs a = base_args(r, B);
  a.q = q;
  a.q_out = q;
  a.m = m;
  a.v = v;
  a.loss = loss;
  a.terms = terms;
  a.dq = dq;
  a.adam = adam_consts(t, lr, b1, b2, eps);
  if (B < kOrderMinB) order = nullptr;
  a.order = order;
  const TileCfg tc = tile_for(ctx, r, B);
  DeviceGuard g(ctx->device);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (order) e = launch_order(q, r.hand.n_dof, B, r.sdf, order, s);
  if (e == hipSuccess) e = launch_step(a, STEP_FUSED, true, tc, s);
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_step_fused_static launch");
  return GRASP_OK;
}

grasp_status grasp_plain_workspace_bytes(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                         const grasp_step_params* p, int32_t B, size_t* out) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!out) return fail(GRASP_EINVAL, "out is NULL");
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  if (r.prm.K != 1) return fail(GRASP_EINVAL, "the plain form runs one projection iteration (K = 1)");
  *out = plain_workspace_floats(r.hand, B) * sizeof(float);
  return GRASP_OK;
}

grasp_status grasp_plain_step(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                              int32_t B, float* q, float* m, float* v, int32_t t, float lr, float b1, float b2,
                              float eps, float* loss, float* terms, void* ws, size_t ws_bytes, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  if (r.prm.K != 1) return fail(GRASP_EINVAL, "the plain form runs one projection iteration (K = 1)");
  if (r.prm.mu > 0.0f) return fail(GRASP_EINVAL, "the plain form has no friction (mu must be 0)");
  if (B > 0 && (!q || !m || !v || !loss || !ws)) return fail(GRASP_EINVAL, "q/m/v/loss/ws is NULL");
  st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  if (ws_bytes < plain_workspace_floats(r.hand, B) * sizeof(float))
    return fail(GRASP_ENOMEM, "workspace too small for the plain form");
  if (reinterpret_cast<uintptr_t>(ws) % 64 != 0) return fail(GRASP_EINVAL, "workspace must be 64-byte aligned");
  DeviceGuard g(ctx->device);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  float* dq = nullptr;
  hipError_t e = launch_plain_step(r.hand, r.sdf, r.prm, B, q, loss, terms, static_cast<float*>(ws), &dq, s);
  if (e == hipSuccess) e = launch_adam(B * r.hand.n_dof, q, m, v, dq, adam_consts(t, lr, b1, b2, eps), s);
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_plain_step launch");
  return GRASP_OK;
}

}  // extern "C"

namespace grasp {
// Checks one batch job and resolves its hand and grid (used by batch.cpp).
grasp_status resolve_job(grasp_ctx* ctx, const grasp_batch_job& j, HandView* h, SdfView* s, StepConsts* c,
                         bool gs_ok) {
  if (j.B < 1 || !j.q || !j.m || !j.v) return fail(GRASP_EINVAL, "batch job needs B >= 1 and q, m, v");
  if (j.t < 0 || j.T < 1 || !(j.r0 >= 0.0f) || !std::isfinite(j.r0)) return fail(GRASP_EINVAL, "bad job schedule");
  grasp_status st = check_adam(j.t + 1, j.lr, j.b1, j.b2, j.eps);
  if (st != GRASP_OK) return st;
  Resolved r;
  st = resolve(ctx, j.hand, j.sdf, &j.p, j.B, &r, gs_ok);
  if (st != GRASP_OK) return st;
  *h = r.hand;
  *s = r.sdf;
  *c = r.prm;
  return GRASP_OK;
}

grasp_status step_fused_gs(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                           int32_t B, float* q, float* m, float* v, int32_t t, float lr, float b1, float b2, float eps,
                           float* loss, float* starts, int* nonfinite, hipStream_t s) {
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r, true);
  if (st != GRASP_OK) return st;
  if (p->projection != GRASP_PROJECTION_GAUSS_SEIDEL) return fail(GRASP_EINVAL, "not a Gauss-Seidel step");
  if (B > 0 && (!q || !m || !v || !starts)) return fail(GRASP_EINVAL, "q/m/v/starts is NULL");
  st = check_adam(t, lr, b1, b2, eps);
  if (st != GRASP_OK) return st;
  StepArgs a = base_args(r, B);
  a.q = q;
  a.q_out = q;
  a.m = m;
  a.v = v;
  a.loss = loss;
  a.nonfinite = nonfinite;
  a.adam = adam_consts(t, lr, b1, b2, eps);
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_gs_step(a, STEP_FUSED, true, starts, s);
  return e == hipSuccess ? GRASP_OK : device_fail(ctx, e, "Gauss-Seidel job step");
}
}  // namespace grasp

extern "C" {

grasp_status grasp_set_tile(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                            int32_t B, const grasp_tile* tile) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (!tile) return fail(GRASP_EINVAL, "tile is NULL");
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  const TileCfg c{tile->waves_per_block, tile->min_waves_per_simd};
  if (!valid_tile(c)) return fail(GRASP_EINVAL, "tile must have waves_per_block in {1,2,4} and min_waves_per_simd in 1..6");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tiles[shape_key(r, B)] = c;
  return GRASP_OK;
}

grasp_status grasp_tune(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                        int32_t B, const float* q, int32_t reps, grasp_tile* best, float* best_ms) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  if (B < 1 || !q || reps < 1) return fail(GRASP_EINVAL, "tune needs B >= 1, q and reps >= 1");
  const size_t nq = static_cast<size_t>(B) * r.hand.n_dof * sizeof(float);
  void* blk = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    blk = ctx->arena.alloc(3 * nq + 256);
  }
  if (!blk) return fail(GRASP_ENOMEM, "arena full (tuning scratch)");
  char* b = static_cast<char*>(blk);
  float* sq = reinterpret_cast<float*>(b);
  float* sm = reinterpret_cast<float*>(b + nq);
  float* sv = reinterpret_cast<float*>(b + 2 * nq);
  DeviceGuard g(ctx->device);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipStreamCreate(&s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  StepArgs a = base_args(r, B);
  a.q = sq;
  a.q_out = sq;
  a.m = sm;
  a.v = sv;
  a.adam = adam_consts(1, 1e-3f, 0.9f, 0.999f, 1e-8f);
  TileCfg bestc{};
  float bestt = 1e30f;
  for (int wpb : {1, 2, 4}) {
    for (int occ = 1; occ <= 6 && e == hipSuccess; ++occ) {
      const TileCfg c{wpb, occ};
      e = hipMemcpyAsync(sq, q, nq, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemsetAsync(sm, 0, 2 * nq, s);
      if (e == hipSuccess) e = launch_ordered_step(ctx, a, STEP_FUSED, true, c, s);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_ordered_step(ctx, a, STEP_FUSED, true, c, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms / reps < bestt) {
        bestt = ms / reps;
        bestc = c;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->arena.free(blk);
    if (e == hipSuccess) ctx->tiles[shape_key(r, B)] = bestc;
  }
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_tune");
  save_tile(shape_key(r, B), bestc);
  if (best) {
    best->waves_per_block = bestc.wpb;
    best->min_waves_per_simd = bestc.occ;
  }
  if (best_ms) *best_ms = bestt;
  return GRASP_OK;
}

grasp_status grasp_debug_sdf_sample(grasp_ctx* ctx, grasp_sdf_id sdf, int32_t n, const float* r, float* out,
                                    float* hess, void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  if (n < 0 || (n > 0 && (!r || !out))) return fail(GRASP_EINVAL, "bad n / NULL r or out");
  SdfView sv;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevSdf* s = find_sdf(ctx, sdf);
    if (!s) return fail(GRASP_EINVAL, "unknown sdf id");
    sv = s->view;
  }
  DeviceGuard g(ctx->device);
  hipError_t e = launch_sample_points(sv, n, r, out, hess, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_debug_sdf_sample launch");
  return GRASP_OK;
}

grasp_status grasp_debug_trace(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                               int32_t B, const float* q, float* p_world, float* poses, float* samples,
                               void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  if (B > 0 && !q) return fail(GRASP_EINVAL, "q is NULL");
  StepArgs a = base_args(r, B);
  a.q = q;
  a.trace_p = p_world;
  a.trace_poses = poses;
  a.trace_samples = samples;
  DeviceGuard g(ctx->device);
  hipError_t e = launch_step(a, STEP_FWD, false, TileCfg{1, 1}, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_debug_trace launch");
  return GRASP_OK;
}

grasp_status grasp_debug_forward_groups(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                        const grasp_step_params* p, int32_t B, const float* q, uint64_t* groups,
                                        void* hip_stream) {
  set_error("");
  GRASP_CHECK_CTX(ctx);
  Resolved r;
  grasp_status st = resolve(ctx, hand, sdf, p, B, &r);
  if (st != GRASP_OK) return st;
  if (!groups) return fail(GRASP_EINVAL, "groups is NULL");
  if (B > 0 && !q) return fail(GRASP_EINVAL, "q is NULL");
  StepArgs a = base_args(r, B);
  a.q = q;
  a.fwd_groups = reinterpret_cast<unsigned long long*>(groups);
  const TileCfg tc = tile_for(ctx, r, B);
  DeviceGuard g(ctx->device);
  hipError_t e = launch_step(a, STEP_FUSED, false, tc, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_debug_forward_groups launch");
  return GRASP_OK;
}

}  // extern "C"

