// Serving loop: continuous batching of render and latent-optimisation
// requests over one pooled sphere tracer.
//
// One persistent ray pool holds the rays of every admitted request.  Each
// tick replays a captured hipGraph on the server stream:
//     clear counters -> apply level changes -> advance (previous active list
//     + coarse-to-fine splits + newly started images -> next active list)
//     -> march (the bf16 decoder on every active ray of every request)
// so requests of different resolutions share every decoder launch, and a
// request that arrives while others are marching joins at the next tick.
// Between ticks the scheduler thread reads the per-image active counts,
// finalises finished requests (maps, normals), and for latent-optimisation
// requests computes the loss, the paper's approximate gradient (adjoint) and
// an Adam step before restarting their images in the pool.
//
// Admission is limited by free ray slots, image/latent slots and the
// context's HBM budget (request buffers are charged against it); a request
// waits in the queue until resources free up.  The queue, tickets, admission
// bookkeeping, the coarse-to-fine tick table and the completion / failure /
// cancellation paths are the device-independent core in sched_core.h; this
// file is its HIP backend (pool, captured tick, per-request buffers, outputs,
// loss, gradient and optimiser step).
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "ray_kernels.h"
#include "sched_core.h"
#include "serve.h"

namespace dist {

int validate_params_ext(const dist_trace_params* p, int H, int W);
int validate_camera_ext(const dist_camera& c, const dist_trace_params* p);
void fill_desc_ext(ImgDesc& d, const dist_camera& c, const dist_trace_params* p, int latent, int slot_base,
                   int out_base);

struct Request : sched::Job {
  dist_request req{};
  std::vector<dist_camera> cams;
  // device buffers of this request (one block from the server cache)
  char* mem = nullptr;
  size_t mem_bytes = 0;
  int* d_imgs = nullptr;
  float *d_depth = nullptr, *d_sil = nullptr, *d_gd = nullptr, *d_gs = nullptr, *d_gz = nullptr, *d_loss = nullptr;
  float* d_fv = nullptr;
  float4* d_nraw = nullptr;
  int *d_hits = nullptr, *d_hit_count = nullptr;
  BwdSpace bw;
};

struct Server : sched::Backend {
  dist_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  std::unique_ptr<sched::Core> core;
  // pool
  int cap_rays = 0, cap_imgs = 0, cap_lat = 0;
  char* mem = nullptr;
  size_t mem_bytes = 0;
  RayPool pool{};
  ImgDesc* imgs = nullptr;
  int* lists[2] = {nullptr, nullptr};
  int* counters = nullptr;       // [2]
  AdvEntry* table = nullptr;
  int* hdr = nullptr;            // [0] entries, [1] new rays
  int* img_active = nullptr;
  unsigned long long* qcount = nullptr;
  int* ecount = nullptr;         // per image slot: queries that returned a non-finite f
  float *z_pool = nullptr, *bias0 = nullptr, *biasS = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  // pinned staging
  AdvEntry* h_table = nullptr;
  int* h_hdr = nullptr;
  int* h_active = nullptr;
  unsigned long long* h_q = nullptr;
  int* h_err = nullptr;
  ImgDesc* h_desc = nullptr;
  float* h_loss = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int parity = 0;
  int adv_grid = 1024;
  // request buffer cache (size -> blocks), charged against the budget
  std::multimap<size_t, char*> cache;

  // the scheduler core's device steps (scheduler thread only)
  bool acquire(sched::Job* j) override;
  void release(sched::Job* j) override;
  void begin(sched::Job* j) override;
  int tick(const std::vector<sched::TickEntry>& table, int n_new) override;
  int active(int img) const override { return h_active[img]; }
  int64_t queries(int img) const override { return (int64_t)h_q[img]; }
  void complete(sched::Job* j) override;
  void settle(sched::Job* j) override;
  void drop_rays() override;
  void thread_init() override { (void)hipSetDevice(ctx->device); }
};

static size_t ray_bytes() {
  return sizeof(float4) + sizeof(float2) + sizeof(int) + 2 + sizeof(float) + kMaxK * (4 + 4 + 1);
}

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
static size_t round_block(size_t b) {
  const size_t g = b < (1u << 20) ? 4096 : (1u << 20);
  return (b + g - 1) / g * g;
}

static int buf_get(Server* s, size_t bytes, char** out) {
  bytes = round_block(bytes);
  auto it = s->cache.find(bytes);
  if (it != s->cache.end()) {
    *out = it->second;
    s->cache.erase(it);
    return DIST_OK;
  }
  void* p = nullptr;
  int rc = ctx_alloc(s->ctx, &p, bytes);
  if (rc == DIST_ENOMEM && !s->cache.empty()) {
    (void)hipStreamSynchronize(s->st);
    for (auto& kv : s->cache) ctx_free(s->ctx, kv.second, kv.first);
    s->cache.clear();
    rc = ctx_alloc(s->ctx, &p, bytes);
  }
  if (rc) return rc;
  *out = (char*)p;
  return DIST_OK;
}

static void buf_put(Server* s, char* p, size_t bytes) {
  if (p) s->cache.emplace(round_block(bytes), p);
}

// ---------------------------------------------------------------------------
// pool set-up and the captured tick
// ---------------------------------------------------------------------------
template <class T>
static T* carve(char*& p, size_t n) {
  p = (char*)(((uintptr_t)p + 255) & ~(uintptr_t)255);
  T* r = (T*)p;
  p += sizeof(T) * n;
  return r;
}

static size_t pool_layout(Server* s, char* base) {
  char* p = base;
  const size_t cap = s->cap_rays;
  RayPool pl{};
  pl.d = carve<float4>(p, cap);
  pl.b = carve<float2>(p, cap);
  pl.img = carve<int>(p, cap);
  pl.st = carve<uint8_t>(p, cap);
  pl.n = carve<uint8_t>(p, cap);
  pl.flast = carve<float>(p, cap);
  pl.rec_f = carve<float>(p, cap * kMaxK);
  pl.rec_t = carve<float>(p, cap * kMaxK);
  pl.rec_n = carve<uint8_t>(p, cap * kMaxK);
  pl.cap = (int)cap;
  s->pool = pl;
  s->imgs = carve<ImgDesc>(p, s->cap_imgs);
  s->lists[0] = carve<int>(p, cap);
  s->lists[1] = carve<int>(p, cap);
  s->counters = carve<int>(p, 4);
  s->table = carve<AdvEntry>(p, s->cap_imgs);
  s->hdr = carve<int>(p, 4);
  s->img_active = carve<int>(p, s->cap_imgs);
  s->qcount = carve<unsigned long long>(p, s->cap_imgs);
  s->ecount = carve<int>(p, s->cap_imgs);
  const int L = s->ctx->L;
  s->z_pool = carve<float>(p, (size_t)s->cap_lat * L);
  s->bias0 = carve<float>(p, (size_t)s->cap_lat * kMaxWidth);
  s->biasS = carve<float>(p, (size_t)s->cap_lat * kMaxWidth);
  s->adam_m = carve<float>(p, (size_t)s->cap_lat * L);
  s->adam_v = carve<float>(p, (size_t)s->cap_lat * L);
  return (size_t)(p - base) + 256;
}

static int capture_tick(Server* s, int par) {
  dist_ctx* ctx = s->ctx;
  const int cur = par, nxt = par ^ 1;
  HIPCHK_S(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
  launch_fill_i32(s->counters + nxt, 0, 1, s->st);
  launch_fill_i32(s->img_active, 0, s->cap_imgs, s->st);
  launch_apply_levels(s->imgs, s->table, s->hdr, s->cap_imgs, s->st);
  launch_advance(s->pool, s->imgs, s->lists[cur], s->counters + cur, s->lists[nxt], s->counters + nxt, s->table,
                 s->hdr, s->img_active, s->adv_grid, s->st);
  MarchArgs ma{};
  ma.net = ctx->net[kPrecBF16];
  ma.pool = s->pool;
  ma.imgs = s->imgs;
  ma.bias0_lat = s->bias0;
  ma.biasS_lat = s->biasS;
  ma.list = s->lists[nxt];
  ma.count = s->counters + nxt;
  ma.qcount = s->qcount;          // queries counted where they are made
  ma.ecount = s->ecount;          // and non-finite ones
  launch_march(kPrecBF16, ma, ctx->n_cu, s->st);
  hipGraph_t g = nullptr;
  HIPCHK_S(hipStreamEndCapture(s->st, &g));
  HIPCHK_S(hipGraphInstantiate(&s->exec[par], g, nullptr, nullptr, 0));
  (void)hipGraphDestroy(g);
  return DIST_OK;
}

static int pool_init(Server* s) {
  dist_ctx* ctx = s->ctx;
  HIPCHK_S(hipSetDevice(ctx->device));
  HIPCHK_S(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
  s->cap_imgs = 4096;
  s->cap_lat = 1024;
  long long cap = 1LL << 25;
  if (ctx->budget) cap = std::min<long long>(cap * 2, (long long)(ctx->budget / 4 / ray_bytes()));
  s->cap_rays = (int)std::max<long long>(cap, 1 << 16);
  s->mem_bytes = pool_layout(s, nullptr);
  void* p = nullptr;
  int rc = ctx_alloc(ctx, &p, s->mem_bytes);
  if (rc) return rc;
  s->mem = (char*)p;
  pool_layout(s, s->mem);
  HIPCHK_S(hipMemsetAsync(s->mem, 0, s->mem_bytes, s->st));
  HIPCHK_S(hipHostMalloc((void**)&s->h_table, sizeof(AdvEntry) * s->cap_imgs));
  HIPCHK_S(hipHostMalloc((void**)&s->h_hdr, sizeof(int) * 4));
  HIPCHK_S(hipHostMalloc((void**)&s->h_active, sizeof(int) * s->cap_imgs));
  HIPCHK_S(hipHostMalloc((void**)&s->h_q, sizeof(unsigned long long) * s->cap_imgs));
  HIPCHK_S(hipHostMalloc((void**)&s->h_err, sizeof(int) * s->cap_imgs));
  HIPCHK_S(hipHostMalloc((void**)&s->h_desc, sizeof(ImgDesc) * s->cap_imgs));
  HIPCHK_S(hipHostMalloc((void**)&s->h_loss, sizeof(float) * s->cap_lat));
  HIPCHK_S(hipStreamSynchronize(s->st));
  for (int par = 0; par < 2; ++par) {
    rc = capture_tick(s, par);
    if (rc) return rc;
  }
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// per-request buffers
// ---------------------------------------------------------------------------
static size_t req_layout(Server* s, Request* r, char* base) {
  char* p = base;
  const size_t npx = (size_t)r->n_views * r->hw;
  r->d_imgs = carve<int>(p, r->n_views);
  r->d_depth = carve<float>(p, npx);
  r->d_sil = carve<float>(p, npx);
  r->d_hits = carve<int>(p, npx);
  r->d_hit_count = carve<int>(p, 4);
  r->d_fv = carve<float>(p, npx * 6);
  r->d_nraw = carve<float4>(p, npx);
  r->d_loss = carve<float>(p, r->n_views + 1);
  if (r->req.kind == DIST_REQ_ZOPT) {
    const int tile = adj_tile_rows(kPrecSplit);
    const int K = r->req.prm.k_samples;
    r->d_gd = carve<float>(p, npx);
    r->d_gs = carve<float>(p, npx);
    r->d_gz = carve<float>(p, (size_t)s->cap_lat * s->ctx->L);
    BwdSpace& b = r->bw;
    b.tile = tile;
    b.cap_samples = (int)(npx * (K + 6) + tile);
    b.cap_blocks = r->n_views * ((r->hw + 255) / 256);
    b.cap_lat = s->cap_lat;
    const int grid = std::max(1, std::min<int>((b.cap_samples + tile - 1) / tile, s->ctx->n_cu));
    b.mask_words = adj_mask_words(kPrecSplit, s->ctx->net[kPrecSplit]) * grid;
    b.samples = carve<float4>(p, b.cap_samples);
    b.sample_lat = carve<int>(p, b.cap_samples);
    b.partial = carve<float>(p, (size_t)(b.cap_samples / tile + 1) * 4 * kMaxWidth);
    b.bsum = carve<int>(p, b.cap_blocks);
    b.boff = carve<int>(p, b.cap_blocks);
    b.seg_base = carve<int>(p, b.cap_lat);
    b.seg_total = carve<int>(p, b.cap_lat);
    b.seg_padded = carve<int>(p, b.cap_lat);
    b.n_samples = carve<int>(p, 4);
    b.mask_ws = carve<unsigned>(p, b.mask_words);
  }
  return (size_t)(p - base) + 256;
}

// Device buffers of a request: one block from the cache, carved.
bool Server::acquire(sched::Job* j) {
  Request* r = static_cast<Request*>(j);
  r->mem_bytes = req_layout(this, r, nullptr);
  if (buf_get(this, r->mem_bytes, &r->mem) != DIST_OK) return false;
  req_layout(this, r, r->mem);
  return true;
}

void Server::release(sched::Job* j) {
  Request* r = static_cast<Request*>(j);
  buf_put(this, r->mem, r->mem_bytes);
  r->mem = nullptr;
}

// Fold the request's latent into the pooled per-latent biases: the start of
// every render (the first, and each z-opt iteration's).
static void fold_latent(Server* s, Request* r) {
  const int L = s->ctx->L;
  const float* z = s->z_pool + (size_t)r->lat * L;
  launch_fold_bias(s->ctx->bf[0], s->ctx->w0z, z, 1, L, s->ctx->out_dims[0], s->ctx->wpad[0],
                   s->bias0 + (size_t)r->lat * s->ctx->wpad[0], s->st);
  if (s->ctx->skip >= 0)
    launch_fold_bias(s->ctx->bf[s->ctx->skip], s->ctx->wsz, z, 1, L, s->ctx->out_dims[s->ctx->skip],
                     s->ctx->wpad[s->ctx->skip], s->biasS + (size_t)r->lat * s->ctx->wpad[s->ctx->skip], s->st);
}

// The request holds its ray slots, image slots and latent slot: descriptors,
// latent code, optimiser state, first render.
void Server::begin(sched::Job* j) {
  Request* r = static_cast<Request*>(j);
  for (int v = 0; v < r->n_views; ++v) {
    ImgDesc& d = h_desc[r->imgs[v]];
    fill_desc_ext(d, r->cams[v], &r->req.prm, r->lat, r->slot_base + v * r->spi, v * r->hw);
    (void)hipMemcpyAsync(imgs + r->imgs[v], &d, sizeof(ImgDesc), hipMemcpyHostToDevice, st);
  }
  (void)hipMemcpyAsync(r->d_imgs, r->imgs.data(), sizeof(int) * r->n_views, hipMemcpyHostToDevice, st);
  for (int v = 0; v < r->n_views; ++v) {
    launch_fill_u64(qcount + r->imgs[v], 1, st);
    launch_fill_i32(ecount + r->imgs[v], 0, 1, st);
  }
  const int L = ctx->L;
  (void)hipMemcpyAsync(z_pool + (size_t)r->lat * L, r->req.z, sizeof(float) * L, hipMemcpyDeviceToDevice, st);
  launch_fill_i32((int*)(adam_m + (size_t)r->lat * L), 0, L, st);
  launch_fill_i32((int*)(adam_v + (size_t)r->lat * L), 0, L, st);
  // the synchronisation below makes the pinned descriptors reusable
  (void)hipStreamSynchronize(st);
  fold_latent(this, r);
}

// Outputs, normals and (z-opt) loss + gradient + Adam for a finished render.
void Server::complete(sched::Job* j) {
  Request* r = static_cast<Request*>(j);
  Server* s = this;
  const dist_request& q = r->req;
  const bool zopt = q.kind == DIST_REQ_ZOPT;
  const bool last = !zopt || r->iter + 1 >= q.iters;
  FinalizeOut fo{};
  fo.depth = (last && q.depth) ? q.depth : r->d_depth;
  fo.sil = (last && q.sil) ? q.sil : r->d_sil;
  fo.status = last ? q.status : nullptr;
  const bool normals = last && q.normal && q.prm.want_normals;
  fo.normal = normals ? q.normal : nullptr;
  fo.nraw = r->d_nraw;
  fo.hits = r->d_hits;
  fo.hit_count = r->d_hit_count;
  fo.want_hits = normals ? 1 : 0;
  launch_fill_i32(r->d_hit_count, 0, 1, s->st);
  launch_finalize(s->pool, s->imgs, r->d_imgs, r->n_views, r->hw, fo, s->st);
  if (normals) {
    EvalArgs ea{};
    ea.net = ctx->net[kPrecSplit];
    ea.bias0_lat = s->bias0;
    ea.biasS_lat = s->biasS;
    ea.mode = 1;
    ea.hits = r->d_hits;
    ea.hit_count = r->d_hit_count;
    ea.pool = s->pool;
    ea.imgs = s->imgs;
    ea.delta = q.prm.normal_delta;
    ea.f_out = r->d_fv;
    const long long rows = 6LL * r->n_views * r->hw;
    launch_eval(kPrecSplit, ea, (int)std::max(1LL, std::min<long long>((rows + 63) / 64, ctx->n_cu)), s->st);
    launch_normals(s->pool, s->imgs, r->d_hits, r->d_hit_count, r->n_views * r->hw, r->d_fv, q.prm.normal_delta,
                   q.normal, r->d_nraw, s->st);
  }
  // a query of this render returned a non-finite f: the request ends with
  // DIST_ENUMERIC (its maps show the rays as DIST_ERROR; no optimiser step)
  for (int img : r->imgs)
    if (h_err[img] > 0) r->error = DIST_ENUMERIC;
  if (!zopt || r->error != DIST_OK) {
    r->finished = true;
    return;
  }
  // loss and its gradient on the maps (depth L1 + silhouette hinge), per
  // view in a fixed order, then summed over the views in view order
  launch_render_loss(fo.depth, nullptr, fo.sil, q.target_depth, nullptr, q.target_sil, r->n_views, r->hw, q.w_depth,
                     q.w_sil, 0.f, r->d_loss, r->d_gd, nullptr, r->d_gs, s->st);
  launch_sum_ordered(r->d_loss, r->n_views, r->d_loss + r->n_views, s->st);
  // gradient samples of this request's images and the adjoint
  BwdSpace& b = r->bw;
  SeedIn in{};
  in.g_depth = r->d_gd;
  in.g_sil = r->d_gs;
  in.nraw = r->d_nraw;
  in.delta = q.prm.normal_delta;
  // image order = view order; all images carry the request's latent slot
  launch_samples(s->pool, s->imgs, r->d_imgs, nullptr, r->n_views, r->hw, s->cap_lat, b.tile, in, b.bsum, b.boff,
                 b.seg_base, b.seg_total, b.seg_padded, b.n_samples, b.samples, b.sample_lat, s->st, r->lat);
  AdjArgs aa{};
  aa.net = ctx->net[kPrecSplit];
  aa.bias0_lat = s->bias0;
  aa.biasS_lat = s->biasS;
  aa.samples = b.samples;
  aa.sample_lat = b.sample_lat;
  aa.n_samples = b.n_samples;
  aa.mask_ws = b.mask_ws;
  aa.partial = b.partial;
  const int grid = std::max(1, std::min<int>((b.cap_samples + b.tile - 1) / b.tile, ctx->n_cu));
  launch_adjoint(kPrecSplit, aa, grid, s->st);
  const int w0 = ctx->wpad[0];
  const int ws = ctx->skip >= 0 ? ctx->wpad[ctx->skip] : 0;
  const int aw = adjoint_waves();
  launch_gz_reduce(b.partial, ctx->kmax, b.tile, b.cap_samples / b.tile + 1, b.seg_base, b.seg_padded, 1, w0,
                   mlp_row_groups(aw, w0), ctx->w0z, ws, ws ? mlp_row_groups(aw, ws) : 1,
                   ctx->skip >= 0 ? ctx->wsz : nullptr, ctx->L, r->d_gz, s->st, r->lat);
  const int L = ctx->L;
  launch_adam(s->z_pool + (size_t)r->lat * L, s->adam_m + (size_t)r->lat * L, s->adam_v + (size_t)r->lat * L,
              r->d_gz + (size_t)r->lat * L, L, q.lr, 0.9f, 0.999f, 1e-8f, r->iter + 1, s->st);
  // the loss reaches the host with the next synchronisation of the server
  // stream (every tick and finish() synchronise); no wait here
  (void)hipMemcpyAsync(s->h_loss + r->lat, r->d_loss + r->n_views, sizeof(float), hipMemcpyDeviceToHost, s->st);
  r->iter += 1;
  if (r->iter >= q.iters) {
    (void)hipMemcpyAsync(q.z_out, s->z_pool + (size_t)r->lat * L, sizeof(float) * L, hipMemcpyDeviceToDevice, s->st);
    r->finished = true;
  } else {
    r->restart();
    fold_latent(s, r);
  }
}

// The request's device work has drained; a z-opt request's last loss is on
// the host.
void Server::settle(sched::Job* j) {
  Request* r = static_cast<Request*>(j);
  (void)hipStreamSynchronize(st);
  if (r->req.kind == DIST_REQ_ZOPT && r->lat >= 0 && r->iter > 0) r->final_loss = h_loss[r->lat];
}

// One tick: the table of images that start rays, the captured graph (clear
// counters, apply level changes, advance, march), then the per-image active
// and query counts back on the host.
int Server::tick(const std::vector<sched::TickEntry>& tab, int n_new) {
  const int n_tab = (int)tab.size();
  for (int i = 0; i < n_tab; ++i) {
    const sched::TickEntry& t = tab[i];
    h_table[i] = AdvEntry{t.img, t.lvl, t.step, t.split, t.begin, t.count};
  }
  h_hdr[0] = n_tab;
  h_hdr[1] = n_new;
  if (n_tab) (void)hipMemcpyAsync(table, h_table, sizeof(AdvEntry) * n_tab, hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(hdr, h_hdr, sizeof(int) * 2, hipMemcpyHostToDevice, st);
  hipError_t e = hipGraphLaunch(exec[parity], st);
  parity ^= 1;
  (void)hipMemcpyAsync(h_active, img_active, sizeof(int) * cap_imgs, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h_q, qcount, sizeof(unsigned long long) * cap_imgs, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h_err, ecount, sizeof(int) * cap_imgs, hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  return (e != hipSuccess || e2 != hipSuccess) ? DIST_EHIP : DIST_OK;
}

void Server::drop_rays() {
  launch_fill_i32(counters, 0, 2, st);
  (void)hipStreamSynchronize(st);
}

}  // namespace dist

using namespace dist;

void serve_shutdown(dist_ctx* ctx) {
  Server* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    s = ctx->server;
    ctx->server = nullptr;
  }
  if (!s) return;
  // jobs still queued or running end DIST_ECANCELLED; then the core and every
  // request it still holds go
  s->core->shutdown();
  (void)hipStreamSynchronize(s->st);
  s->core.reset();
  for (int p = 0; p < 2; ++p)
    if (s->exec[p]) (void)hipGraphExecDestroy(s->exec[p]);
  for (auto& kv : s->cache) ctx_free(ctx, kv.second, kv.first);
  if (s->mem) ctx_free(ctx, s->mem, s->mem_bytes);
  (void)hipHostFree(s->h_table);
  (void)hipHostFree(s->h_hdr);
  (void)hipHostFree(s->h_active);
  (void)hipHostFree(s->h_q);
  (void)hipHostFree(s->h_err);
  (void)hipHostFree(s->h_desc);
  (void)hipHostFree(s->h_loss);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

static Server* get_server(dist_ctx* ctx, int* rc) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  if (ctx->server) return ctx->server;
  Server* s = new Server();
  s->ctx = ctx;
  *rc = pool_init(s);
  if (*rc) {
    if (s->mem) ctx_free(ctx, s->mem, s->mem_bytes);
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return nullptr;
  }
  s->core.reset(new sched::Core(s, s->cap_rays, s->cap_imgs, s->cap_lat, 4096));
  s->core->start();
  ctx->server = s;
  return s;
}

extern "C" int dist_submit(dist_ctx* ctx, const dist_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket) return dist_set_error(DIST_EINVAL, "null argument");
  if (ctx->n_out != 1) return dist_set_error(DIST_EINVAL, "a colour network does not render geometry");
  if (req->kind != DIST_REQ_RENDER && req->kind != DIST_REQ_ZOPT) return dist_set_error(DIST_EINVAL, "bad kind");
  if (req->n_views < 1 || req->n_views > 64 || !req->cams) return dist_set_error(DIST_EINVAL, "n_views in [1, 64]");
  if (!req->z) return dist_set_error(DIST_EINVAL, "null latent code");
  if (req->prm.precision != DIST_BF16)
    return dist_set_error(DIST_EINVAL, "serving marches pooled rays with the bf16 decoder (precision DIST_BF16)");
  const int H = req->cams[0].H, W = req->cams[0].W;
  for (int v = 0; v < req->n_views; ++v) {
    if (req->cams[v].H != H || req->cams[v].W != W) return dist_set_error(DIST_EINVAL, "views must share H, W");
    int rc = validate_camera_ext(req->cams[v], &req->prm);
    if (rc) return rc;
  }
  int rc = validate_params_ext(&req->prm, H, W);
  if (rc) return rc;
  if (req->kind == DIST_REQ_ZOPT) {
    if (!req->target_depth || !req->target_sil || !req->z_out || req->iters < 1)
      return dist_set_error(DIST_EINVAL, "z-opt needs targets, z_out and iters >= 1");
    if (!(req->lr > 0.f)) return dist_set_error(DIST_EINVAL, "lr must be positive");
  }
  Server* s = get_server(ctx, &rc);
  if (!s) return rc ? rc : dist_set_error(DIST_EHIP, "server start failed");
  Request* r = new Request();
  r->req = *req;
  r->cams.assign(req->cams, req->cams + req->n_views);
  r->req.cams = r->cams.data();
  r->kind = req->kind;
  r->H = H;
  r->W = W;
  r->hw = H * W;
  r->n_views = req->n_views;
  r->levels = req->prm.c2f_levels;
  r->spi = slots_per_image(r->hw, r->levels);
  r->max_steps = req->prm.max_steps;
  r->iters = req->kind == DIST_REQ_ZOPT ? req->iters : 1;
  if ((long long)r->n_views * r->spi > s->cap_rays) {
    delete r;
    return dist_set_error(DIST_ENOMEM, "request needs more ray slots than the pool holds");
  }
  const size_t need = round_block(req_layout(s, r, nullptr));
  if (ctx->budget && need + s->mem_bytes > ctx->budget) {
    delete r;
    return dist_set_error(DIST_ENOMEM, "request can never fit the HBM budget (%zu bytes needed)", need);
  }
  rc = s->core->submit(r, ticket);
  if (rc == DIST_EBUSY) return dist_set_error(DIST_EBUSY, "serving queue full");
  if (rc) return dist_set_error(rc, "the server is shutting down");
  return DIST_OK;
}

extern "C" int dist_poll(dist_ctx* ctx, uint64_t ticket, dist_result* res, int64_t timeout_us) {
  if (!ctx || !res) return dist_set_error(DIST_EINVAL, "null argument");
  Server* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    s = ctx->server;
  }
  if (!s) return dist_set_error(DIST_ENOTFOUND, "unknown ticket");
  const int rc = s->core->poll(ticket, res, timeout_us);
  if (rc == DIST_ENOTFOUND) return dist_set_error(DIST_ENOTFOUND, "unknown ticket");
  return rc;
}
