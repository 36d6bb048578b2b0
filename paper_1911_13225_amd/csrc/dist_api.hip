// Host side of the C ABI (include/dist.h): validation, packed weights,
// workspaces and the launch sequence of the forward and backward passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "dist.h"
#include "dist_internal.h"
#include "ray_kernels.h"
#include "ctx.h"
#include "serve.h"

using namespace dist;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int dist_set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return dist_set_error(DIST_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

extern "C" const char* dist_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// scratch of the allocation-free decoder query (dist_sdf_eval_noalloc): the
// per-latent folded biases live in this array instead of a workspace.  Each
// GPU holds its own copy for the life of the process.  Host code must never
// pass `scratch` itself to a kernel (on the host it is only a stand-in
// symbol): its device address is taken once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchFloats = size_t(1) << 18;   // 1 MiB per GPU
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxScratchDevices] = {};

// Resolve the scratch address on `device`, which must be the current device.
static int scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices)
    return dist_set_error(DIST_EINVAL, "device %d is beyond the %d devices the scratch table covers", device,
                          kMaxScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return DIST_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return dist_set_error(DIST_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                          hipGetErrorString(e));
  g_scratch_ptr[device] = (float*)ptr;
  return DIST_OK;
}

extern "C" const char* dist_version(void) { return "dist-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static int pad_width(int w) { return w <= 128 ? 128 : (w <= 256 ? 256 : 512); }

int ctx_alloc(dist_ctx* ctx, void** p, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  {
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    if (ctx->budget && ctx->used + bytes > ctx->budget)
      return dist_set_error(DIST_ENOMEM, "allocation of %zu bytes exceeds the HBM budget (%zu of %zu used)", bytes,
                            ctx->used, ctx->budget);
    ctx->used += bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    ctx->used -= bytes;
    return dist_set_error(DIST_EHIP, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return DIST_OK;
}

void ctx_free(dist_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  bytes = (bytes + 255) & ~(size_t)255;
  (void)hipFree(p);
  std::lock_guard<std::mutex> lk(ctx->mem_mu);
  ctx->used -= bytes;
}

static int pack_weights(dist_ctx* ctx, const float* const* W, const float* const* b, hipStream_t st) {
  const int nl = ctx->nl, L = ctx->L, skip = ctx->skip;
  // float32 master copies
  for (int l = 0; l < nl; ++l) {
    HIPCHK(hipMemcpyAsync(ctx->Wf[l], W[l], sizeof(float) * ctx->out_dims[l] * ctx->in_dims[l],
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->bf[l], b[l], sizeof(float) * ctx->out_dims[l], hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  // host copies of the small pieces
  std::vector<float> W0(ctx->out_dims[0] * ctx->in_dims[0]);
  HIPCHK(hipMemcpy(W0.data(), W[0], W0.size() * 4, hipMemcpyDeviceToHost));
  const int w0 = ctx->wpad[0];
  std::vector<float> w0p(3 * w0, 0.f), w0z((size_t)w0 * L, 0.f);
  for (int n = 0; n < ctx->out_dims[0]; ++n) {
    for (int j = 0; j < L; ++j) w0z[(size_t)n * L + j] = W0[(size_t)n * ctx->in_dims[0] + j];
    for (int a = 0; a < 3; ++a) w0p[a * w0 + n] = W0[(size_t)n * ctx->in_dims[0] + L + a];
  }
  HIPCHK(hipMemcpy(ctx->w0p, w0p.data(), w0p.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->w0z, w0z.data(), w0z.size() * 4, hipMemcpyHostToDevice));
  if (skip >= 0) {
    const int ws = ctx->wpad[skip], nh = ctx->out_dims[skip - 1], in = ctx->in_dims[skip];
    std::vector<float> Ws((size_t)ctx->out_dims[skip] * in);
    HIPCHK(hipMemcpy(Ws.data(), W[skip], Ws.size() * 4, hipMemcpyDeviceToHost));
    std::vector<float> wsp(3 * ws, 0.f), wsz((size_t)ws * L, 0.f);
    for (int n = 0; n < ctx->out_dims[skip]; ++n) {
      for (int j = 0; j < L; ++j) wsz[(size_t)n * L + j] = Ws[(size_t)n * in + nh + j];
      for (int a = 0; a < 3; ++a) wsp[a * ws + n] = Ws[(size_t)n * in + nh + L + a];
    }
    HIPCHK(hipMemcpy(ctx->wsp, wsp.data(), wsp.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->wsz, wsz.data(), wsz.size() * 4, hipMemcpyHostToDevice));
  }
  // padded biases of hidden layers
  for (int l = 0; l < nl - 1; ++l) {
    std::vector<float> bb(ctx->wpad[l], 0.f);
    HIPCHK(hipMemcpy(bb.data(), b[l], ctx->out_dims[l] * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ctx->bias_pad[l], bb.data(), bb.size() * 4, hipMemcpyHostToDevice));
  }
  // output layer: n_out rows, each padded to the last hidden width
  {
    const int lo = nl - 1, no = ctx->n_out, wp = ctx->wpad[nl - 2], in = ctx->in_dims[lo];
    std::vector<float> Wl((size_t)no * in), wl((size_t)no * wp, 0.f), bl(no, 0.f);
    HIPCHK(hipMemcpy(Wl.data(), W[lo], Wl.size() * 4, hipMemcpyDeviceToHost));
    for (int c = 0; c < no; ++c)
      for (int k = 0; k < in; ++k) wl[(size_t)c * wp + k] = Wl[(size_t)c * in + k];
    HIPCHK(hipMemcpy(ctx->wlast, wl.data(), wl.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bl.data(), b[lo], no * 4, hipMemcpyDeviceToHost));
    for (int p = 0; p < 3; ++p) {
      ctx->net[p].blast = bl[0];
      for (int c = 0; c < 3; ++c) ctx->net[p].blast_c[c] = c < no ? bl[c] : 0.f;
    }
  }
  // MFMA fragments
  for (int l = 1; l <= nl - 2; ++l) {
    const int out = ctx->out_dims[l], in = ctx->in_dims[l];
    const int ncols = (l == skip) ? ctx->out_dims[l - 1] : in;
    for (int p = 0; p < 2; ++p) {
      launch_pack_w(p, false, ctx->Wf[l], out, in, ncols, ctx->wpad[l], ctx->kpad[l], ctx->wpack[p][l], st);
      launch_pack_w(p, true, ctx->Wf[l], out, in, ncols, ctx->wpad[l], ctx->kpad[l], ctx->wpackT[p][l], st);
    }
    launch_pack_w(kPrecSplit, false, ctx->Wf[l], out, in, ncols, ctx->wpad[l], ctx->kpad[l], ctx->wpacklo[l], st);
    for (int q = 0; q < 2; ++q) launch_pack_bias(q, ctx->bias_pad[l], ctx->wpad[l], ctx->bfrag[q][l], st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return DIST_OK;
}

extern "C" int dist_create(dist_ctx** out, const dist_decoder_desc* desc, const float* const* W,
                           const float* const* b, size_t hbm_budget_bytes, void* stream) {
  if (!out || !desc || !W || !b || !desc->out_dims) return dist_set_error(DIST_EINVAL, "null argument");
  const int nl = desc->n_layers, L = desc->latent_dim, skip = desc->skip_layer;
  if (nl < 3 || nl > kMaxLayers) return dist_set_error(DIST_EINVAL, "n_layers must be in [3, %d]", kMaxLayers);
  if (L < 1 || L > 512) return dist_set_error(DIST_EINVAL, "latent_dim must be in [1, 512]");
  if (skip != -1 && (skip < 1 || skip >= nl - 2))
    return dist_set_error(DIST_EINVAL, "skip_layer must be -1 or in [1, n_layers-3]");
  if (desc->out_dims[nl - 1] != 1 && desc->out_dims[nl - 1] != 3)
    return dist_set_error(DIST_EINVAL, "the last layer must have width 1 (signed distance) or 3 (colour)");
  for (int l = 0; l < nl - 1; ++l)
    if (desc->out_dims[l] < 1 || desc->out_dims[l] > kMaxWidth)
      return dist_set_error(DIST_EINVAL, "hidden widths must be in [1, %d]", kMaxWidth);
  for (int l = 0; l < nl; ++l)
    if (!W[l] || !b[l]) return dist_set_error(DIST_EINVAL, "null weight pointer for layer %d", l);
  hipStream_t st = (hipStream_t)stream;

  dist_ctx* ctx = new dist_ctx();
  ctx->n_out = desc->out_dims[nl - 1];
  ctx->nl = nl;
  ctx->L = L;
  ctx->skip = skip;
  ctx->budget = hbm_budget_bytes;
  ctx->out_dims.assign(desc->out_dims, desc->out_dims + nl);
  ctx->in_dims.resize(nl);
  for (int l = 0; l < nl; ++l) {
    ctx->in_dims[l] = (l == 0) ? L + 3 : ctx->out_dims[l - 1] + ((l == skip) ? L + 3 : 0);
  }
  if (hipGetDevice(&ctx->device) != hipSuccess) { delete ctx; return dist_set_error(DIST_EHIP, "no HIP device"); }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || ncu <= 0)
    ncu = 256;
  ctx->n_cu = ncu;
  ctx->wpad.assign(nl, 0);
  ctx->kpad.assign(nl, 0);
  int kmax = 0;
  for (int l = 0; l < nl - 1; ++l) {
    ctx->wpad[l] = pad_width(ctx->out_dims[l]);
    kmax = std::max(kmax, ctx->wpad[l]);
  }
  for (int l = 1; l <= nl - 2; ++l) ctx->kpad[l] = ctx->wpad[l - 1];
  ctx->kmax = kmax;

  int rc = DIST_OK;
  auto A = [&](void** p, size_t bytes) {
    if (rc == DIST_OK) {
      rc = ctx_alloc(ctx, p, bytes);
      if (rc == DIST_OK) ctx->owned.push_back({*p, bytes});
    }
  };
  ctx->Wf.assign(nl, nullptr);
  ctx->bf.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    A((void**)&ctx->Wf[l], sizeof(float) * ctx->out_dims[l] * ctx->in_dims[l]);
    A((void**)&ctx->bf[l], sizeof(float) * ctx->out_dims[l]);
  }
  A((void**)&ctx->w0p, sizeof(float) * 3 * ctx->wpad[0]);
  A((void**)&ctx->w0z, sizeof(float) * ctx->wpad[0] * L);
  if (skip >= 0) {
    A((void**)&ctx->wsp, sizeof(float) * 3 * ctx->wpad[skip]);
    A((void**)&ctx->wsz, sizeof(float) * ctx->wpad[skip] * L);
  }
  ctx->bias_pad.assign(nl, nullptr);
  for (int l = 0; l < nl - 1; ++l) A((void**)&ctx->bias_pad[l], sizeof(float) * ctx->wpad[l]);
  A((void**)&ctx->wlast, sizeof(float) * ctx->wpad[nl - 2] * ctx->n_out);
  for (int p = 0; p < 2; ++p) {
    ctx->wpack[p].assign(nl, nullptr);
    ctx->wpackT[p].assign(nl, nullptr);
    const size_t es = p ? 2 : 4;
    for (int l = 1; l <= nl - 2; ++l) {
      A(&ctx->wpack[p][l], es * ctx->wpad[l] * ctx->kpad[l]);
      A(&ctx->wpackT[p][l], es * ctx->wpad[l] * ctx->kpad[l]);
    }
  }
  ctx->wpacklo.assign(nl, nullptr);
  for (int l = 1; l <= nl - 2; ++l) A(&ctx->wpacklo[l], 2 * ctx->wpad[l] * ctx->kpad[l]);
  for (int q = 0; q < 2; ++q) {
    ctx->bfrag[q].assign(nl, nullptr);
    for (int l = 1; l <= nl - 2; ++l) A(&ctx->bfrag[q][l], (size_t)(ctx->wpad[l] / 32) * 64 * (q ? 16 : 4));
  }
  if (rc != DIST_OK) { dist_destroy(ctx); return rc; }
  for (int p = 0; p < 3; ++p) {
    const int q = p == 0 ? 0 : 1;      // split precision shares the bf16 packs (hi parts)
    NetDev& nd = ctx->net[p];
    memset(&nd, 0, sizeof nd);
    nd.nl = nl;
    nd.L = L;
    nd.skip = skip;
    nd.kmax = kmax;
    for (int l = 0; l < nl; ++l) {
      nd.wpad[l] = ctx->wpad[l];
      nd.kpad[l] = ctx->kpad[l];
      nd.wp[l] = ctx->wpack[q][l];
      nd.wpT[l] = ctx->wpackT[q][l];
      nd.wplo[l] = p == 2 ? ctx->wpacklo[l] : nullptr;
      nd.bias[l] = ctx->bias_pad[l];
      nd.bfrag[l] = ctx->bfrag[q][l];
    }
    nd.w0p = ctx->w0p;
    nd.wsp = ctx->wsp;
    nd.wlast = ctx->wlast;
    nd.nout = ctx->n_out;
  }
  rc = pack_weights(ctx, W, b, st);
  if (rc == DIST_OK) {
    for (int p = 0; p < 3; ++p) {
      hipError_t e = mlp_setup(p, ctx->net[p]);
      if (e != hipSuccess) {
        rc = dist_set_error(DIST_EHIP, "raising the LDS limit failed: %s", hipGetErrorString(e));
        break;
      }
    }
  }
  if (rc == DIST_OK) rc = scratch_setup(ctx->device);
  if (rc != DIST_OK) { dist_destroy(ctx); return rc; }
  *out = ctx;
  return DIST_OK;
}

extern "C" int dist_set_weights(dist_ctx* ctx, const float* const* W, const float* const* b, void* stream) {
  if (!ctx || !W || !b) return dist_set_error(DIST_EINVAL, "null argument");
  for (int l = 0; l < ctx->nl; ++l)
    if (!W[l] || !b[l]) return dist_set_error(DIST_EINVAL, "null weight pointer for layer %d", l);
  return pack_weights(ctx, W, b, (hipStream_t)stream);
}

static void ws_release_all(dist_ctx* ctx);

extern "C" int dist_destroy(dist_ctx* ctx) {
  if (!ctx) return dist_set_error(DIST_EINVAL, "null context");
  serve_shutdown(ctx);
  (void)hipDeviceSynchronize();
  ws_release_all(ctx);
  for (int k = 0; k < kTimeClasses; ++k)
    for (auto& pr : ctx->tev[k]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  if (ctx->col) {
    if (ctx->col->bw) {
      ctx_free(ctx, ctx->col->bw->mem, ctx->col->bw->bytes);
      delete ctx->col->bw;
    }
    ctx_free(ctx, ctx->col->mem, ctx->col->bytes);
    delete ctx->col;
  }
  if (ctx->theta) {
    ctx_free(ctx, ctx->theta->mem, ctx->theta->bytes);
    delete ctx->theta;
  }
  for (auto& o : ctx->owned) ctx_free(ctx, o.first, o.second);
  delete ctx;
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
__global__ void k_acc_rows(const int* rows, int mul, unsigned long long* acc) {
  if (threadIdx.x == 0) *acc += (unsigned long long)(*rows) * (unsigned long long)mul;
}

TimedLaunch::TimedLaunch(dist_ctx* c, int kk, hipStream_t s, const int* rows, int mul) : ctx(c), k(kk), st(s) {
  if (!ctx->timing) return;
  if (rows && ctx->d_rows) hipLaunchKernelGGL(k_acc_rows, dim3(1), dim3(64), 0, st, rows, mul, ctx->d_rows + k);
  auto& v = ctx->tev[k];
  if (ctx->tev_used[k] == v.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    v.push_back({a, b});
  }
  auto& pr = v[ctx->tev_used[k]++];
  (void)hipEventRecord(pr.first, st);
  end = pr.second;
}

TimedLaunch::~TimedLaunch() {
  if (end) (void)hipEventRecord(end, st);
}

extern "C" int dist_timing_enable(dist_ctx* ctx, int on) {
  if (!ctx) return dist_set_error(DIST_EINVAL, "null context");
  HIPCHK(hipDeviceSynchronize());
  if (!ctx->d_rows) {
    int rc = ctx_alloc(ctx, (void**)&ctx->d_rows, kTimeClasses * sizeof(unsigned long long));
    if (rc) return rc;
    ctx->owned.push_back({ctx->d_rows, kTimeClasses * sizeof(unsigned long long)});
  }
  HIPCHK(hipMemset(ctx->d_rows, 0, kTimeClasses * sizeof(unsigned long long)));
  HIPCHK(hipDeviceSynchronize());
  ctx->timing = on != 0;
  for (int k = 0; k < kTimeClasses; ++k) ctx->tev_used[k] = 0;
  return DIST_OK;
}

extern "C" int dist_timing_read(dist_ctx* ctx, int32_t kernel, dist_kernel_time* out) {
  if (!ctx || !out || kernel < 0 || kernel >= kTimeClasses) return dist_set_error(DIST_EINVAL, "bad argument");
  double ms = 0.0;
  for (size_t i = 0; i < ctx->tev_used[kernel]; ++i) {
    auto& pr = ctx->tev[kernel][i];
    HIPCHK(hipEventSynchronize(pr.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
    ms += t;
  }
  unsigned long long rows = 0;
  if (ctx->d_rows) HIPCHK(hipMemcpy(&rows, ctx->d_rows + kernel, sizeof rows, hipMemcpyDeviceToHost));
  out->launches = (int64_t)ctx->tev_used[kernel];
  out->ms = ms;
  out->rows = (int64_t)rows;
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// workspaces: one device allocation carved into the buffers of a render
// ---------------------------------------------------------------------------
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(base ? base + off : nullptr);
    off += sizeof(T) * count;
    return p;
  }
};

static void ws_layout(Workspace& w, Carver& c) {
  const size_t cap = w.cap_rays;
  w.pool.d = c.take<float4>(cap);
  w.pool.b = c.take<float2>(cap);
  w.pool.img = c.take<int>(cap);
  w.pool.st = c.take<uint8_t>(cap);
  w.pool.n = c.take<uint8_t>(cap);
  w.pool.flast = c.take<float>(cap);
  w.pool.rec_f = c.take<float>(cap * kMaxK);
  w.pool.rec_t = c.take<float>(cap * kMaxK);
  w.pool.rec_n = c.take<uint8_t>(cap * kMaxK);
  w.pool.cap = (int)cap;
  w.imgs = c.take<ImgDesc>(w.cap_img);
  w.imgs_list = c.take<int>(w.cap_img);
  w.img_order = c.take<int>(w.cap_img);
  w.img_latent = c.take<int>(w.cap_img);
  w.list[0] = c.take<int>(cap);
  w.list[1] = c.take<int>(cap);
  w.counters = c.take<int>(w.cap_steps + 8);
  w.qcount = c.take<unsigned long long>(w.cap_img);
  w.bias0_lat = c.take<float>((size_t)w.cap_lat * kMaxWidth);
  w.biasS_lat = c.take<float>((size_t)w.cap_lat * kMaxWidth);
  w.hits = c.take<int>(w.cap_pix);
  w.fv = c.take<float>((size_t)w.cap_pix * 6);
  w.nraw = c.take<float4>(w.cap_pix);
  w.hit_pix = c.take<int>(w.cap_pix);
  w.img_view = c.take<int>(w.cap_img);
}

static void bw_layout(BwdSpace& w, Carver& c) {
  w.samples = c.take<float4>(w.cap_samples);
  w.sample_lat = c.take<int>(w.cap_samples);
  w.partial = c.take<float>((size_t)(w.cap_samples / w.tile + 1) * 4 * kMaxWidth);
  w.bsum = c.take<int>(w.cap_blocks);
  w.boff = c.take<int>(w.cap_blocks);
  w.seg_base = c.take<int>(w.cap_lat);
  w.seg_total = c.take<int>(w.cap_lat);
  w.seg_padded = c.take<int>(w.cap_lat);
  w.n_samples = c.take<int>(4);
  w.mask_ws = c.take<unsigned>(w.mask_words);
  w.bsum2 = c.take<int>(w.cap_blocks);
  w.boff2 = c.take<int>(w.cap_blocks);
  w.seg2_base = c.take<int>(w.cap_lat);
  w.seg2_total = c.take<int>(w.cap_lat);
  w.seg2_padded = c.take<int>(w.cap_lat);
  w.sample_idx = c.take<int>(w.cap_samples);
  w.partial2 = c.take<float>((size_t)(w.cap_samples / w.tile + 1) * 4 * kMaxWidth);
}

static int ws_get(dist_ctx* ctx, int cap_rays, int cap_pix, int cap_img, int cap_lat, int cap_steps,
                  Workspace** out) {
  {
    std::lock_guard<std::mutex> lk(ctx->ws_mu);
    for (size_t i = 0; i < ctx->ws_free.size(); ++i) {
      Workspace* w = ctx->ws_free[i];
      if (w->cap_rays >= cap_rays && w->cap_pix >= cap_pix && w->cap_img >= cap_img && w->cap_lat >= cap_lat &&
          w->cap_steps >= cap_steps) {
        ctx->ws_free.erase(ctx->ws_free.begin() + i);
        *out = w;
        return DIST_OK;
      }
    }
  }
  Workspace* w = new Workspace();
  w->cap_rays = cap_rays;
  w->cap_pix = cap_pix;
  w->cap_img = cap_img;
  w->cap_lat = cap_lat;
  w->cap_steps = cap_steps;
  Carver c;
  ws_layout(*w, c);
  w->bytes = c.off + 256;
  int rc = ctx_alloc(ctx, (void**)&w->mem, w->bytes);
  if (rc != DIST_OK) {
    // free cached workspaces and retry once
    ws_release_all(ctx);
    rc = ctx_alloc(ctx, (void**)&w->mem, w->bytes);
    if (rc != DIST_OK) { delete w; return rc; }
  }
  c.base = w->mem;
  c.off = 0;
  ws_layout(*w, c);
  if (hipHostMalloc((void**)&w->h_imgs, sizeof(ImgDesc) * cap_img) != hipSuccess ||
      hipHostMalloc((void**)&w->h_ints, sizeof(int) * 4 * cap_img) != hipSuccess ||
      hipEventCreateWithFlags(&w->staged, hipEventDisableTiming) != hipSuccess) {
    ctx_free(ctx, w->mem, w->bytes);
    delete w;
    return dist_set_error(DIST_EHIP, "pinned staging allocation failed");
  }
  w->staged_pending = false;
  *out = w;
  return DIST_OK;
}

void ws_put(dist_ctx* ctx, Workspace* w) {
  std::lock_guard<std::mutex> lk(ctx->ws_mu);
  ctx->ws_free.push_back(w);
}

static void ws_destroy(dist_ctx* ctx, Workspace* w) {
  if (w->staged_pending) (void)hipEventSynchronize(w->staged);
  (void)hipEventDestroy(w->staged);
  (void)hipHostFree(w->h_imgs);
  (void)hipHostFree(w->h_ints);
  ctx_free(ctx, w->mem, w->bytes);
  if (w->bw) {
    ctx_free(ctx, w->bw->mem, w->bw->bytes);
    delete w->bw;
  }
  if (w->ns) {
    ctx_free(ctx, w->ns->mem, w->ns->bytes);
    delete w->ns;
  }
  if (w->cs) {
    ctx_free(ctx, w->cs->mem, w->cs->bytes);
    delete w->cs;
  }
  if (w->us) {
    ctx_free(ctx, w->us->mem, w->us->bytes);
    delete w->us;
  }
  if (w->gs) {
    ctx_free(ctx, w->gs->mem, w->gs->bytes);
    delete w->gs;
  }
  delete w;
}

static void ws_release_all(dist_ctx* ctx) {
  std::vector<Workspace*> v;
  {
    std::lock_guard<std::mutex> lk(ctx->ws_mu);
    v.swap(ctx->ws_free);
  }
  if (!v.empty()) (void)hipDeviceSynchronize();
  for (Workspace* w : v) ws_destroy(ctx, w);
}

static int bw_get_into(dist_ctx* ctx, BwdSpace*& slot, int cap_samples, int cap_blocks, int cap_lat, int tile,
                       size_t mask_words) {
  BwdSpace* b = slot;
  if (b && b->cap_samples >= cap_samples && b->cap_blocks >= cap_blocks && b->cap_lat >= cap_lat && b->tile == tile &&
      b->mask_words >= mask_words)
    return DIST_OK;
  if (b) {
    ctx_free(ctx, b->mem, b->bytes);
    delete b;
    slot = nullptr;
  }
  b = new BwdSpace();
  b->cap_samples = cap_samples;
  b->cap_blocks = cap_blocks;
  b->cap_lat = cap_lat;
  b->tile = tile;
  b->mask_words = mask_words;
  Carver c;
  bw_layout(*b, c);
  b->bytes = c.off + 256;
  int rc = ctx_alloc(ctx, (void**)&b->mem, b->bytes);
  if (rc != DIST_OK) { delete b; return rc; }
  c.base = b->mem;
  c.off = 0;
  bw_layout(*b, c);
  slot = b;
  return DIST_OK;
}

static int bw_get(dist_ctx* ctx, Workspace* w, int cap_samples, int cap_blocks, int cap_lat, int tile,
                  size_t mask_words) {
  return bw_get_into(ctx, w->bw, cap_samples, cap_blocks, cap_lat, tile, mask_words);
}

// Buffers for the ReLU masks of up to cap_samples stencil queries.
static int ns_get(dist_ctx* ctx, Workspace* w, long long cap_samples, size_t words) {
  NrmSave* n = w->ns;
  if (n && n->cap_samples >= cap_samples && n->words == words) return DIST_OK;
  if (n) {
    ctx_free(ctx, n->mem, n->bytes);
    delete n;
    w->ns = nullptr;
  }
  n = new NrmSave();
  n->cap_samples = cap_samples;
  n->words = words;
  const size_t mbytes = ((size_t)cap_samples * words * 4 + 255) & ~(size_t)255;
  n->bytes = mbytes + (size_t)cap_samples * 4 + 256;
  int rc = ctx_alloc(ctx, (void**)&n->mem, n->bytes);
  if (rc != DIST_OK) { delete n; return rc; }
  n->mask = (unsigned*)n->mem;
  n->dtanh = (float*)(n->mem + mbytes);
  w->ns = n;
  return DIST_OK;
}

// Scratch of the device grouping of cap_n explicit samples over cap_lat latents.
static int gs_get(dist_ctx* ctx, Workspace* w, int cap_n, int cap_lat) {
  GroupSpace* g = w->gs;
  if (g && g->cap_n >= cap_n && g->cap_lat >= cap_lat) return DIST_OK;
  if (g) {
    ctx_free(ctx, g->mem, g->bytes);
    delete g;
    w->gs = nullptr;
  }
  g = new GroupSpace();
  g->cap_n = std::max(cap_n, 1);
  g->cap_lat = std::max(cap_lat, 1);
  g->temp_bytes = group_temp_bytes(g->cap_n, g->cap_lat);
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t kb = up((size_t)g->cap_n * 4), lb = up((size_t)g->cap_lat * 4);
  g->bytes = 4 * kb + 2 * lb + up(g->temp_bytes);
  int rc = ctx_alloc(ctx, (void**)&g->mem, g->bytes);
  if (rc != DIST_OK) { delete g; return rc; }
  char* m = g->mem;
  g->keys_in = (int*)m;
  g->vals_in = (int*)(m + kb);
  g->keys_out = (int*)(m + 2 * kb);
  g->vals_out = (int*)(m + 3 * kb);
  g->cnt = (int*)(m + 4 * kb);
  g->start = (int*)(m + 4 * kb + lb);
  g->temp = m + 4 * kb + 2 * lb;
  w->gs = g;
  return DIST_OK;
}

// Buffers of the gradient through the unrolled march: t of cap_lam ray slots
// at each of steps steps, and one adjoint per slot.
static int us_get(dist_ctx* ctx, Workspace* w, long long cap_lam, int steps) {
  UnrollSpace* u = w->us;
  const long long cap_hist = cap_lam * steps;
  if (u && u->cap_hist >= cap_hist && u->cap_lam >= cap_lam) return DIST_OK;
  if (u) {
    ctx_free(ctx, u->mem, u->bytes);
    delete u;
    w->us = nullptr;
  }
  u = new UnrollSpace();
  u->cap_hist = cap_hist;
  u->cap_lam = cap_lam;
  const size_t hb = ((size_t)cap_hist * 4 + 255) & ~(size_t)255;
  u->bytes = hb + (size_t)cap_lam * 4 + 256;
  int rc = ctx_alloc(ctx, (void**)&u->mem, u->bytes);
  if (rc != DIST_OK) { delete u; return rc; }
  u->t_hist = (float*)u->mem;
  u->lam = (float*)(u->mem + hb);
  w->us = u;
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// forward render
// ---------------------------------------------------------------------------
static int validate_params(const dist_trace_params* p, int H, int W) {
  if (!(p->alpha > 0.f) || !(p->eps > 0.f) || !(p->normal_delta > 0.f))
    return dist_set_error(DIST_EINVAL, "alpha, eps and normal_delta must be positive");
  if (p->max_steps < 1 || p->max_steps > 255) return dist_set_error(DIST_EINVAL, "max_steps must be in [1, 255]");
  if (p->c2f_levels < 0 || p->c2f_levels > 2) return dist_set_error(DIST_EINVAL, "c2f_levels must be 0, 1 or 2");
  if (p->max_steps <= 3 * p->c2f_levels)
    return dist_set_error(DIST_EINVAL, "max_steps must exceed 3 * c2f_levels");
  if (p->k_samples < 1 || p->k_samples > kMaxK) return dist_set_error(DIST_EINVAL, "k_samples must be in [1, 4]");
  if (p->precision != DIST_FP32 && p->precision != DIST_BF16 && p->precision != DIST_BF16X3)
    return dist_set_error(DIST_EINVAL, "precision must be DIST_FP32, DIST_BF16 or DIST_BF16X3");
  if (p->keep_history != 0 && p->keep_history != 1) return dist_set_error(DIST_EINVAL, "keep_history must be 0 or 1");
  const int m = 1 << p->c2f_levels;
  if (H < 1 || W < 1 || H % m || W % m || (long long)H * W > (1 << 22))
    return dist_set_error(DIST_EINVAL, "H and W must be positive multiples of 2^c2f_levels (at most 4M pixels)");
  return DIST_OK;
}

static int validate_camera(const dist_camera& c, const dist_trace_params* p) {
  const double r = std::sqrt((double)c.c[0] * c.c[0] + (double)c.c[1] * c.c[1] + (double)c.c[2] * c.c[2]);
  if (!(r > 1.0)) return dist_set_error(DIST_EINVAL, "camera centre must lie outside the unit sphere");
  if (!(p->near_ <= r - 1.0) || !(p->far_ >= r + 1.0))
    return dist_set_error(DIST_EINVAL, "near/far must not clip the unit sphere (near <= |c|-1, far >= |c|+1)");
  if (!(c.fx > 0.f) || !(c.fy > 0.f)) return dist_set_error(DIST_EINVAL, "focal lengths must be positive");
  return DIST_OK;
}

static void fill_desc(ImgDesc& d, const dist_camera& c, const dist_trace_params* p, int latent, int slot_base,
                      int out_base) {
  memset(&d, 0, sizeof d);
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  for (int i = 0; i < 9; ++i) d.R[i] = c.R_wc[i];
  for (int i = 0; i < 3; ++i) d.c[i] = c.c[i];
  d.alpha = p->alpha; d.eps = p->eps; d.near_ = p->near_; d.far_ = p->far_;
  d.H = c.H; d.W = c.W; d.levels = p->c2f_levels; d.latent = latent;
  d.max_steps = p->max_steps; d.K = p->k_samples; d.cur_level = p->c2f_levels;
  d.slot_base = slot_base;
  const int hw = c.H * c.W;
  d.lvl_off[0] = 0;
  d.lvl_off[1] = hw;
  d.lvl_off[2] = hw + hw / 4;
  d.out_base = out_base;
}

namespace dist {
int validate_params_ext(const dist_trace_params* p, int H, int W) { return validate_params(p, H, W); }
int validate_camera_ext(const dist_camera& c, const dist_trace_params* p) { return validate_camera(c, p); }
void fill_desc_ext(ImgDesc& d, const dist_camera& c, const dist_trace_params* p, int latent, int slot_base,
                   int out_base) {
  fill_desc(d, c, p, latent, slot_base, out_base);
}
}  // namespace dist

int slots_per_image(int hw, int levels) {
  int s = 0;
  for (int l = 0; l <= levels; ++l) s += hw >> (2 * l);
  // keep the level offsets of fill_desc valid whatever the level count
  return std::max(s, hw + hw / 4 + (levels >= 2 ? hw / 16 : 0));
}

// Stage image descriptors and the per-image index arrays (pinned -> device).
static int stage_images(Workspace* w, const std::vector<ImgDesc>& d, const std::vector<int>& order,
                        const std::vector<int>& lat, const std::vector<int>& view, hipStream_t st) {
  if (w->staged_pending) HIPCHK(hipEventSynchronize(w->staged));
  const int n = (int)d.size();
  memcpy(w->h_imgs, d.data(), sizeof(ImgDesc) * n);
  for (int i = 0; i < n; ++i) {
    w->h_ints[i] = i;
    w->h_ints[n + i] = order[i];
    w->h_ints[2 * n + i] = lat[i];
    w->h_ints[3 * n + i] = view[i];
  }
  HIPCHK(hipMemcpyAsync(w->img_view, w->h_ints + 3 * n, sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w->imgs, w->h_imgs, sizeof(ImgDesc) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w->imgs_list, w->h_ints, sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w->img_order, w->h_ints + n, sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w->img_latent, w->h_ints + 2 * n, sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(w->staged, st));
  w->staged_pending = true;
  return DIST_OK;
}

int fold_biases(dist_ctx* ctx, Workspace* w, const float* z, int n_lat, hipStream_t st) {
  launch_fold_bias(ctx->bf[0], ctx->w0z, z, n_lat, ctx->L, ctx->out_dims[0], ctx->wpad[0], w->bias0_lat, st);
  if (ctx->skip >= 0)
    launch_fold_bias(ctx->bf[ctx->skip], ctx->wsz, z, n_lat, ctx->L, ctx->out_dims[ctx->skip],
                     ctx->wpad[ctx->skip], w->biasS_lat, st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

static int mlp_grid(dist_ctx* ctx, long long rows, int prec) {
  const long long tiles = (rows + mlp_tile_rows(prec) - 1) / mlp_tile_rows(prec);
  return (int)std::max(1LL, std::min<long long>(tiles, ctx->n_cu));
}

// March all images of a workspace from their coarsest level to completion.
int run_trace(dist_ctx* ctx, Workspace* w, int n_img, int hw, const dist_trace_params* prm, hipStream_t st,
              float* t_hist) {
  const int L = prm->c2f_levels, prec = prm->precision;
  launch_fill_i32(w->counters, 0, prm->max_steps + 8, st);
  launch_fill_u64(w->qcount, n_img, st);
  launch_init_level(w->pool, w->imgs, w->imgs_list, n_img, hw >> (2 * L), w->list[0], w->counters, st);
  MarchArgs ma{};
  ma.net = ctx->net[prec];
  ma.pool = w->pool;
  ma.imgs = w->imgs;
  ma.bias0_lat = w->bias0_lat;
  ma.biasS_lat = w->biasS_lat;
  ma.qcount = w->qcount;
  ma.t_hist = t_hist;
  // steps before the last coarse-to-fine split: one launch per step, every
  // image splitting after the same steps
  int* tail_cnt = w->counters + prm->max_steps + 5;
  for (int n = 0; n < 3 * L; ++n) {
    const int lv = L - n / 3;
    const long long rays = (long long)n_img * (hw >> (2 * lv));
    ma.list = w->list[n & 1];
    ma.count = w->counters + n;
    // at a split the children replace the rays, otherwise the march step
    // appends its survivors to the next list
    const bool split = n % 3 == 2;
    int* nxt = w->list[(n + 1) & 1];
    int* ncnt = w->counters + n + 1;
    ma.next_list = split ? nullptr : nxt;
    ma.next_count = split ? nullptr : ncnt;
    {
      TimedLaunch tl(ctx, 0, st, ma.count, 1);
      // the bf16 march may choose 64-row tiles, so size its grid by those
      launch_march(prec, ma, mlp_grid(ctx, rays, prec == kPrecBF16 ? kPrecSplit : prec), st);
    }
    // the last split orders the full-resolution list for the one-launch
    // march: children of rays still marching first, the others from the
    // list's end
    if (split)
      launch_split(w->pool, w->imgs, w->imgs_list, n_img, hw >> (2 * (lv - 1)), lv - 1, n + 1, nxt, ncnt, st,
                   lv == 1 ? tail_cnt : nullptr, w->pool.cap);
  }
  // full resolution: every remaining step in one launch; the rays of the
  // step's list are claimed into per-workgroup rings carved from the other
  // list (grid and ring size bounded by its capacity)
  {
    const int n = 3 * L;
    const long long cap = w->pool.cap;
    const int grid = (int)std::max(1LL, std::min<long long>(ctx->n_cu, cap / 256));
    ma.list = w->list[n & 1];
    ma.count = w->counters + n;
    ma.count_tail = L > 0 ? tail_cnt : nullptr;
    ma.tail_end = w->pool.cap;
    ma.next_list = w->list[(n + 1) & 1];
    ma.next_count = nullptr;
    ma.claim = w->counters + n + 1;
    ma.ring_cap = (int)std::min<long long>(4096, cap / grid);
    ma.rows_done = (ctx->timing && ctx->d_rows) ? ctx->d_rows + 0 : nullptr;
    TimedLaunch tl(ctx, 0, st);
    launch_march_ring(prec, ma, grid, st);
  }
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

// Finalise outputs and compute normals with float32 queries.
int run_finalize(dist_ctx* ctx, Workspace* w, int n_img, int hw, const dist_trace_params* prm, float* depth,
                 float* dist, float* normal, float* sil, uint8_t* status, uint8_t* nsteps, hipStream_t st,
                 bool keep_masks) {
  FinalizeOut fo{};
  fo.depth = depth;
  fo.dist = dist;
  fo.sil = sil;
  fo.normal = normal;
  fo.status = status;
  fo.nsteps = nsteps;
  fo.nraw = w->nraw;
  fo.hits = w->hits;
  fo.hit_count = w->counters + prm->max_steps + 4;
  fo.want_hits = prm->want_normals ? 1 : 0;
  fo.hit_pix = keep_masks ? w->hit_pix : nullptr;
  launch_fill_i32(fo.hit_count, 0, 1, st);
  launch_finalize(w->pool, w->imgs, nullptr, n_img, hw, fo, st);
  if (prm->want_normals) {
    // normal queries: float32, or split bf16 (float32-class accuracy) on the bf16 paths
    const int np = prm->precision == DIST_FP32 ? kPrecF32 : kPrecSplit;
    EvalArgs ea{};
    ea.net = ctx->net[np];
    ea.bias0_lat = w->bias0_lat;
    ea.biasS_lat = w->biasS_lat;
    ea.mode = 1;
    ea.hits = w->hits;
    ea.hit_count = fo.hit_count;
    ea.pool = w->pool;
    ea.imgs = w->imgs;
    ea.delta = prm->normal_delta;
    ea.f_out = w->fv;
    if (keep_masks) {
      ea.mask_out = w->ns->mask;
      ea.dtanh_out = w->ns->dtanh;
    }
    {
      TimedLaunch tl(ctx, 1, st, fo.hit_count, 6);
      launch_eval(np, ea, mlp_grid(ctx, 6LL * n_img * hw, np), st);
    }
    launch_normals(w->pool, w->imgs, w->hits, fo.hit_count, n_img * hw, w->fv, prm->normal_delta, normal, w->nraw,
                   st);
  }
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

__global__ void k_u64_to_i64(const unsigned long long* a, int64_t* b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int64_t)a[i];
}

extern "C" int dist_render_fwd(dist_ctx* ctx, const dist_camera* cams, int32_t n_views, const float* z,
                               int32_t n_latents, const int32_t* pairs, int32_t n_images,
                               const dist_trace_params* prm, float* depth, float* dist, float* normal, float* sil,
                               uint8_t* status, uint8_t* nsteps, int64_t* queries, dist_saved** saved,
                               void* stream) {
  if (!ctx || !cams || !z || !prm) return dist_set_error(DIST_EINVAL, "null argument");
  if (ctx->n_out != 1) return dist_set_error(DIST_EINVAL, "a colour network does not render geometry");
  if (n_views < 1 || n_latents < 1) return dist_set_error(DIST_EINVAL, "n_views and n_latents must be positive");
  const int n_img = pairs ? n_images : n_views * n_latents;
  if (n_img < 1 || n_img > kMaxImages) return dist_set_error(DIST_EINVAL, "n_images must be in [1, %d]", kMaxImages);
  const int H = cams[0].H, W = cams[0].W;
  for (int v = 0; v < n_views; ++v) {
    if (cams[v].H != H || cams[v].W != W) return dist_set_error(DIST_EINVAL, "all views must share H and W");
    int rc = validate_camera(cams[v], prm);
    if (rc) return rc;
  }
  int rc = validate_params(prm, H, W);
  if (rc) return rc;
  std::vector<int> vi(n_img), li(n_img);
  for (int i = 0; i < n_img; ++i) {
    vi[i] = pairs ? pairs[2 * i] : i / n_latents;
    li[i] = pairs ? pairs[2 * i + 1] : i % n_latents;
    if (vi[i] < 0 || vi[i] >= n_views || li[i] < 0 || li[i] >= n_latents)
      return dist_set_error(DIST_EINVAL, "pair %d out of range", i);
  }
  if (saved) *saved = nullptr;
  hipStream_t st = (hipStream_t)stream;
  const int hw = H * W;
  const int spi = slots_per_image(hw, prm->c2f_levels);
  const long long cap_rays = (long long)n_img * spi;
  if (cap_rays > (1LL << 30)) return dist_set_error(DIST_EINVAL, "too many rays in one call");
  Workspace* w = nullptr;
  rc = ws_get(ctx, (int)cap_rays, n_img * hw, n_img, n_latents, prm->max_steps, &w);
  if (rc) return rc;
  std::vector<ImgDesc> d(n_img);
  for (int i = 0; i < n_img; ++i) fill_desc(d[i], cams[vi[i]], prm, li[i], i * spi, i * hw);
  std::vector<int> order(n_img);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return li[a] < li[b]; });
  rc = stage_images(w, d, order, li, vi, st);
  if (!rc) rc = fold_biases(ctx, w, z, n_latents, st);
  // a forward whose state is saved keeps the ReLU masks of its normal-stencil
  // queries, so that the backward skips their recompute
  const int np = prm->precision == DIST_FP32 ? kPrecF32 : kPrecSplit;
  const long long n_stencil = 6LL * n_img * hw;
  const size_t mwords = (size_t)(ctx->nl - 1) * (ctx->net[np].kmax / 32);
  bool keep = saved && prm->want_normals && n_stencil <= INT_MAX && n_stencil * (long long)mwords <= (1LL << 40);
  if (!rc && keep && ns_get(ctx, w, n_stencil, mwords) != DIST_OK) keep = false;  // fall back to the recompute
  // a saved forward asked to keep its march history records t per step
  const bool hist = saved && prm->keep_history;
  if (!rc && hist) rc = us_get(ctx, w, w->pool.cap, prm->max_steps);
  if (!rc) rc = run_trace(ctx, w, n_img, hw, prm, st, hist ? w->us->t_hist : nullptr);
  if (!rc) rc = run_finalize(ctx, w, n_img, hw, prm, depth, dist, normal, sil, status, nsteps, st, keep);
  if (!rc && queries) hipLaunchKernelGGL(k_u64_to_i64, dim3((n_img + 255) / 256), dim3(256), 0, st, w->qcount, queries, n_img);
  if (rc) {
    ws_put(ctx, w);
    return rc;
  }
  if (saved) {
    dist_saved* s = new dist_saved();
    s->ctx = ctx;
    s->ws = w;
    s->n_img = n_img;
    s->hw = hw;
    s->n_lat = n_latents;
    s->n_views = n_views;
    s->prm = *prm;
    s->z = z;
    s->img_latent = li;
    s->order = order;
    s->masks_kept = keep;
    s->hist_kept = hist;
    *saved = s;
  } else {
    ws_put(ctx, w);
  }
  return DIST_OK;
}

extern "C" int dist_saved_free(dist_saved* s) {
  if (!s) return dist_set_error(DIST_EINVAL, "null saved state");
  ws_put(s->ctx, s->ws);
  delete s;
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// The adjoint of a bf16 render recomputes the forward in split precision (the
// ReLU pattern must match the float32 network; a bf16 recompute flips units
// near zero) and back-propagates in bf16.
static int adj_prec(int render_prec) { return render_prec == DIST_FP32 ? kPrecF32 : kPrecSplit; }
// The VJP from saved masks needs no recompute, so on the bf16 paths it runs
// the bf16 kernel (128-row tiles, the same bf16 products as the split
// kernel's VJP, which uses only the hi parts).
static int vjp_prec(int adj) { return adj == kPrecSplit ? kPrecBF16 : adj; }

// Row groups of the column sums S0 and Sskip written by a VJP kernel of `waves` waves.
static int groups_s0(dist_ctx* ctx, int waves) { return mlp_row_groups(waves, ctx->wpad[0]); }
static int groups_skip(dist_ctx* ctx, int waves) {
  return ctx->skip >= 0 ? mlp_row_groups(waves, ctx->wpad[ctx->skip]) : 1;
}

static int reduce_only(dist_ctx* ctx, BwdSpace* b, int n_lat, float* g_z, hipStream_t st) {
  const int w0 = ctx->wpad[0];
  const int ws = ctx->skip >= 0 ? ctx->wpad[ctx->skip] : 0;
  const int aw = adjoint_waves();
  launch_gz_reduce(b->partial, ctx->kmax, b->tile, b->cap_samples / b->tile + 1, b->seg_base, b->seg_padded, n_lat,
                   w0, groups_s0(ctx, aw), ctx->w0z, ws, groups_skip(ctx, aw), ctx->skip >= 0 ? ctx->wsz : nullptr,
                   ctx->L, g_z, st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

static int run_adjoint_and_reduce(dist_ctx* ctx, Workspace* w, BwdSpace* b, int prec, int n_lat, float* g_z,
                                  bool split, hipStream_t st) {
  AdjArgs aa{};
  aa.net = ctx->net[prec];
  aa.bias0_lat = w->bias0_lat;
  aa.biasS_lat = w->biasS_lat;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  const int grid = mlp_grid(ctx, b->cap_samples, prec);
  {
    TimedLaunch tl(ctx, 2, st, b->n_samples, 1);
    launch_adjoint(prec, aa, grid, st);
  }
  if (split) {
    // the normal-stencil samples (second list): VJP from the masks the forward kept
    const int vp = vjp_prec(prec);
    aa.net = ctx->net[vp];
    aa.partial = b->partial2;
    aa.n_begin = b->n_samples;
    aa.n_samples = b->n_samples + 2;
    aa.sample_idx = b->sample_idx;
    aa.smask = w->ns->mask;
    aa.sdtanh = w->ns->dtanh;
    {
      TimedLaunch tl(ctx, 3, st, b->n_samples + 3, 1);
      launch_vjp_saved(vp, aa, mlp_grid(ctx, b->cap_samples, vp), st);
    }
  }
  const int w0 = ctx->wpad[0];
  const int ws = ctx->skip >= 0 ? ctx->wpad[ctx->skip] : 0;
  // every wave covers all rows of a tile, so each column sum has one row group
  const int aw = adjoint_waves();
  launch_gz_reduce(b->partial, ctx->kmax, b->tile, b->cap_samples / b->tile + 1, b->seg_base, b->seg_padded, n_lat,
                   w0, groups_s0(ctx, aw), ctx->w0z, ws, groups_skip(ctx, aw), ctx->skip >= 0 ? ctx->wsz : nullptr,
                   ctx->L, g_z, st);
  if (split) {
    const int vt = adj_tile_rows(vjp_prec(prec));
    const int vw = vjp_saved_waves(vjp_prec(prec));
    launch_gz_reduce(b->partial2, ctx->kmax, vt, b->cap_samples / vt + 1, b->seg2_base, b->seg2_padded, n_lat, w0,
                     groups_s0(ctx, vw), ctx->w0z, ws, groups_skip(ctx, vw), ctx->skip >= 0 ? ctx->wsz : nullptr,
                     ctx->L, g_z, st, 0, 1);
  }
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

__global__ void k_zero_f32(float* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// Weight gradient (Sec. 3.4: dL/dtheta = sum over samples of seed * df/dtheta
// at the detached points).  Per layer, dW_l = sum_rows Delta_l (x) x_l and
// db_l = sum_rows Delta_l, where Delta_l is the row's seed times dm/d(pre-
// activation of layer l) and x_l the layer's input ([h] for hidden layers,
// [z, p] for layer 0, [h, z, p] for the skip layer).  The recompute-and-VJP
// kernel captures h and Delta of every row of a chunk in the blocked
// feature-major layout of the capture (64-row blocks, a block's features
// contiguous; bfloat16 on the bf16 paths, float32 on the float32 path); each layer's
// contraction over the chunk's rows runs on MFMA (one k_dw launch per layer
// and chunk, every input segment and the bias in it).  The contraction is
// long (all samples) and the output small (a layer's weights), so the rows of
// a chunk are cut into slices of kThetaSlice that run in parallel; slice s of
// every chunk adds to its own partial, and one launch per layer sums the
// partials in slice order into g_W / g_b: the sum order is fixed, so the
// result is reproducible bit for bit.  The capture and partial buffers belong
// to the context and are reused; the one host synchronisation reads the
// sample count that sizes the chunk loop.
static constexpr int kThetaChunkRows = 65536;
static constexpr int kThetaSlice = 2048;
static constexpr int kThetaSlices = kThetaChunkRows / kThetaSlice;
static_assert(kThetaSlice % kDwRows == 0, "slices are whole LDS blocks of the contraction");

// g_W[n][k] = sum over slices s (in order) of P[s][n][k] for k < k_in, and
// g_b[n] the same sum of column k_in.
__global__ void k_slice_sum(const float* __restrict__ P, int S, int n_out, int k_in, float* __restrict__ gW,
                            float* __restrict__ gb) {
  const int ldp = k_in + 1;
  const long long total = (long long)n_out * ldp;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int sl = 0; sl < S; ++sl) acc += P[sl * total + i];
    const long long n = i / ldp, k = i - n * ldp;
    if (k < k_in) gW[n * k_in + k] = acc;
    else gb[n] = acc;
  }
}

static size_t theta_partials(const dist_ctx* ctx) {
  size_t f = 0;
  for (int l = 0; l < ctx->nl; ++l) f += (size_t)ctx->out_dims[l] * (ctx->in_dims[l] + 1);
  return f * kThetaSlices;
}

static int theta_space(dist_ctx* ctx, int prec, int rows) {
  ThetaSpace*& t = ctx->theta;
  if (t && t->prec == prec && t->rows >= rows) return DIST_OK;
  if (t) {
    ctx_free(ctx, t->mem, t->bytes);
    delete t;
    t = nullptr;
  }
  const size_t es = prec == kPrecF32 ? 4 : 2;
  const size_t nfeat = (size_t)(ctx->nl - 1) * ctx->kmax;
  const size_t al = 256;
  auto up = [&](size_t x) { return (x + al - 1) / al * al; };
  const size_t hb = up(rows * nfeat * es), gb = up(rows * es), zb = up((size_t)rows * ctx->L * es),
               pb = up((size_t)rows * 4 * es);
  const size_t sb = up(theta_partials(ctx) * 4);
  ThetaSpace* n = new ThetaSpace();
  n->bytes = 2 * hb + 2 * gb + zb + pb + sb;
  int rc = ctx_alloc(ctx, &n->mem, n->bytes);
  if (rc) {
    delete n;
    return rc;
  }
  char* m = (char*)n->mem;
  n->hbuf = (float*)m;
  n->dbuf = (float*)(m + hb);
  n->gmbuf = (float*)(m + 2 * hb);
  n->ones = m + 2 * hb + gb;
  n->zrows = m + 2 * hb + 2 * gb;
  n->prows = m + 2 * hb + 2 * gb + zb;
  n->slices = (float*)(m + 2 * hb + 2 * gb + zb + pb);
  n->rows = rows;
  n->prec = prec;
  t = n;
  return DIST_OK;
}

static int run_theta(dist_ctx* ctx, Workspace* w, BwdSpace* b, int prec, const float* z, float* const* g_W,
                     float* const* g_b, hipStream_t st) {
  for (int l = 0; l < ctx->nl; ++l)
    if (!g_W[l] || !g_b[l]) return dist_set_error(DIST_EINVAL, "null weight-gradient pointer for layer %d", l);
  int ns = 0;
  HIPCHK(hipMemcpyAsync(&ns, b->n_samples, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int tile = b->tile;
  const int tiles = ns / tile;
  if (tiles == 0) {
    for (int l = 0; l < ctx->nl; ++l) {
      hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, st, g_W[l],
                         (long long)ctx->out_dims[l] * ctx->in_dims[l]);
      hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, st, g_b[l], (long long)ctx->out_dims[l]);
    }
    HIPCHK(hipGetLastError());
    return DIST_OK;
  }
  const int chunk = std::max(1, std::min(tiles, kThetaChunkRows / tile));
  // contraction rows per chunk: whole slices (rows past the chunk's samples are zero)
  auto gemm_rows_of = [](int valid) {
    return valid >= kThetaSlice ? (valid + kThetaSlice - 1) / kThetaSlice * kThetaSlice : valid;
  };
  const int R = gemm_rows_of(chunk * tile);
  if (R % kCapBlock != 0 || tile != kCapBlock || (prec != kPrecF32 && R % kDwRows != 0))
    return dist_set_error(DIST_EINVAL, "weight-gradient chunk of %d rows is not whole blocks", R);
  int rc = theta_space(ctx, prec, R);
  if (rc) return rc;
  ThetaSpace* t = ctx->theta;
  const int es = prec == kPrecF32 ? 4 : 2;
  const int kmax = ctx->kmax;
  auto at = [&](const void* base, size_t off) { return (const void*)((const char*)base + off * es); };
  AdjArgs aa{};
  aa.net = ctx->net[prec];
  aa.bias0_lat = w->bias0_lat;
  aa.biasS_lat = w->biasS_lat;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  aa.hbuf = t->hbuf;
  aa.dbuf = t->dbuf;
  aa.gmbuf = t->gmbuf;
  aa.cap_rows = R;
  const int L = ctx->L, nl = ctx->nl;
  // per layer: its partials and the input segments of its contraction
  std::vector<DwArgs> da(nl);
  {
    size_t off = 0;
    for (int l = 0; l < nl; ++l) {
      DwArgs& d = da[l];
      d.D = l < nl - 1 ? at(t->dbuf, (size_t)l * kmax * R) : (const void*)t->gmbuf;
      d.FD = l < nl - 1 ? kmax : 1;
      d.R = R;
      d.n_out = ctx->out_dims[l];
      d.k_in = ctx->in_dims[l];
      d.ldp = d.k_in + 1;
      d.P = t->slices + off;
      off += (size_t)kThetaSlices * d.n_out * d.ldp;
      int e = 0;
      // a segment: its base, the features it contributes and its features per capture block
      auto seg = [&](const void* p, int n, int F) {
        d.x.p[d.x.nseg] = p;
        d.x.F[d.x.nseg] = F;
        e += n;
        d.x.end[d.x.nseg++] = e;
      };
      const int nh = l == 0 ? 0 : ctx->out_dims[l - 1];       // width of the h part of the input
      if (nh > 0) seg(at(t->hbuf, (size_t)(l - 1) * kmax * R), nh, kmax);
      if (l == 0 || l == ctx->skip) {
        seg(t->zrows, L, L);
        seg(t->prows, 3, 4);
      }
      if (prec == kPrecF32) seg(t->ones, 1, 1);
      if (e != d.k_in + (prec == kPrecF32 ? 1 : 0))
        return dist_set_error(DIST_EINVAL, "layer %d input segments cover %d of %d features", l, e, d.k_in);
      d.kcols = e;
      d.bias = prec == kPrecF32 ? 0 : 1;
    }
  }
  int S0 = 0;
  for (int t0 = 0; t0 < tiles; t0 += chunk) {
    const int t1 = std::min(tiles, t0 + chunk);
    const int valid = (t1 - t0) * tile;
    const int rows = gemm_rows_of(valid);
    const int S = rows >= kThetaSlice ? rows / kThetaSlice : 1;
    if (t0 == 0) S0 = S;
    aa.tile_begin = t0;
    aa.tile_end = t1;
    {
      // the rows of every chunk, counted once (all samples)
      TimedLaunch tl(ctx, 2, st, t0 == 0 ? b->n_samples : nullptr, 1);
      launch_adjoint(prec, aa, std::max(1, std::min(t1 - t0, ctx->n_cu)), st);
    }
    launch_theta_rows(prec, b->samples + (size_t)t0 * tile, b->sample_lat + (size_t)t0 * tile, z, L, valid, R,
                      t->zrows, t->prows, t->ones, t->hbuf, t->dbuf, t->gmbuf, nl - 1, kmax, st);
    for (int l = 0; l < nl; ++l) {
      DwArgs d = da[l];
      d.S = S;
      d.K = rows / S;
      d.acc = t0 > 0;
      TimedLaunch tl(ctx, 4, st);
      launch_dw(prec, d, st);
    }
  }
  for (int l = 0; l < nl; ++l) {
    const long long total = (long long)da[l].n_out * da[l].ldp;
    hipLaunchKernelGGL(k_slice_sum, dim3((int)std::min<long long>((total + 255) / 256, 4096)), dim3(256), 0, st,
                       da[l].P, S0, da[l].n_out, da[l].k_in, g_W[l], g_b[l]);
  }
  HIPCHK(hipGetLastError());
  return rc;
}

static int cs_get(dist_ctx* ctx, Workspace* w, long long cap_samples, long long cap_pix = 0) {
  CamSpace* c = w->cs;
  if (c && c->cap_samples >= cap_samples && c->cap_pix >= cap_pix) return DIST_OK;
  cap_samples = std::max(cap_samples, c ? c->cap_samples : 0);
  cap_pix = std::max(cap_pix, c ? c->cap_pix : 0);
  if (c) {
    ctx_free(ctx, c->mem, c->bytes);
    delete c;
    w->cs = nullptr;
  }
  c = new CamSpace();
  c->cap_samples = cap_samples;
  c->cap_pix = cap_pix;
  const size_t a = ((size_t)cap_samples * sizeof(int4) + 255) & ~(size_t)255;
  const size_t g = ((size_t)cap_samples * 3 * kGpSlots * sizeof(float) + 255) & ~(size_t)255;
  c->bytes = a + g + (size_t)cap_pix * sizeof(float) + 256;
  int rc = ctx_alloc(ctx, (void**)&c->mem, c->bytes);
  if (rc != DIST_OK) { delete c; return rc; }
  c->sample_cam = (int4*)c->mem;
  c->gp = (float*)(c->mem + a);
  c->gv = (float*)(c->mem + a + g);
  w->cs = c;
  return DIST_OK;
}

// The backward of dist_render_bwd; with imp_gv the depth term of each hit is
// the exact (implicit-function) one, using grad f . v measured per pixel.
static int render_bwd(dist_ctx* ctx, const dist_saved* saved, const float* g_depth, const float* g_normal,
                      const float* g_sil, float* g_z, float* const* g_W, float* const* g_b, const float* imp_gv,
                      hipStream_t st) {
  Workspace* w = saved->ws;
  const int prec = adj_prec(saved->prm.precision);
  const int tile = adj_tile_rows(prec);
  const int n_img = saved->n_img, hw = saved->hw, n_lat = saved->n_lat;
  // the weight gradient captures every row's activations, so it recomputes the
  // stencil samples too; g_z alone uses the masks the forward kept
  const bool split = saved->masks_kept && !g_W && g_normal != nullptr;
  // sample lists are padded per latent to a multiple of both kernels' tiles
  const int pad = split ? std::max(tile, adj_tile_rows(vjp_prec(prec))) : tile;
  const long long cap = (long long)n_img * hw * (std::max(saved->prm.k_samples, 2) + 6) + 2LL * n_lat * pad;
  if (cap > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many gradient samples");
  const int bpi = (hw + 255) / 256;
  const int grid = mlp_grid(ctx, cap, prec);
  int rc = bw_get(ctx, w, (int)cap, n_img * bpi, n_lat, tile, adj_mask_words(prec, ctx->net[prec]) * grid);
  if (rc) return rc;
  BwdSpace* b = w->bw;
  SeedIn in{};
  in.g_depth = g_depth;
  in.g_normal = saved->prm.want_normals ? g_normal : nullptr;
  in.g_sil = g_sil;
  in.nraw = w->nraw;
  in.delta = saved->prm.normal_delta;
  in.hit_pix = split ? w->hit_pix : nullptr;
  in.imp_gv = imp_gv;
  const SplitList sl{b->bsum2, b->boff2, b->seg2_base, b->seg2_total, b->seg2_padded, b->sample_idx};
  launch_samples(w->pool, w->imgs, w->img_order, w->img_latent, n_img, hw, n_lat, pad, in, b->bsum, b->boff,
                 b->seg_base, b->seg_total, b->seg_padded, b->n_samples, b->samples, b->sample_lat, st, 0,
                 split ? &sl : nullptr);
  HIPCHK(hipGetLastError());
  if (g_W) {
    rc = run_theta(ctx, w, b, prec, saved->z, g_W, g_b, st);
    if (rc) return rc;
    return reduce_only(ctx, b, n_lat, g_z, st);
  }
  return run_adjoint_and_reduce(ctx, w, b, prec, n_lat, g_z, split, st);
}

extern "C" int dist_render_bwd(dist_ctx* ctx, const dist_saved* saved, const float* g_depth, const float* g_normal,
                               const float* g_sil, float* g_z, float* const* g_W, float* const* g_b, void* stream) {
  if (!ctx || !saved || !g_z) return dist_set_error(DIST_EINVAL, "null argument");
  if (saved->ctx != ctx) return dist_set_error(DIST_EINVAL, "saved state belongs to another context");
  if ((g_W == nullptr) != (g_b == nullptr)) return dist_set_error(DIST_EINVAL, "pass both g_W and g_b, or neither");
  return render_bwd(ctx, saved, g_depth, g_normal, g_sil, g_z, g_W, g_b, nullptr, (hipStream_t)stream);
}

__global__ void k_fill_f32(float* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

extern "C" int dist_render_bwd_implicit(dist_ctx* ctx, const dist_saved* saved, const float* g_depth,
                                        const float* g_normal, const float* g_sil, float* g_z, void* stream) {
  if (!ctx || !saved || !g_z) return dist_set_error(DIST_EINVAL, "null argument");
  if (saved->ctx != ctx) return dist_set_error(DIST_EINVAL, "saved state belongs to another context");
  hipStream_t st = (hipStream_t)stream;
  if (!g_depth) return render_bwd(ctx, saved, g_depth, g_normal, g_sil, g_z, nullptr, nullptr, nullptr, st);
  Workspace* w = saved->ws;
  const int prec = adj_prec(saved->prm.precision);
  const int tile = adj_tile_rows(prec);
  const int n_img = saved->n_img, hw = saved->hw, n_lat = saved->n_lat;
  const long long npix = (long long)n_img * hw;
  // pass 1: grad f . v at the Eq. 1 point of every hit with a depth gradient.
  // The buffers are sized for pass 2 up front (no reallocation between passes).
  const int pad = std::max(tile, adj_tile_rows(vjp_prec(prec)));
  const long long cap2 = npix * (std::max(saved->prm.k_samples, 2) + 6) + 2LL * n_lat * pad;
  const long long cap = npix + (long long)n_lat * tile;
  if (cap2 > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many gradient samples");
  const int bpi = (hw + 255) / 256;
  const int grid = mlp_grid(ctx, cap2, prec);
  int rc = bw_get(ctx, w, (int)cap2, n_img * bpi, n_lat, tile, adj_mask_words(prec, ctx->net[prec]) * grid);
  if (!rc) rc = cs_get(ctx, w, cap, npix);
  if (rc) return rc;
  BwdSpace* b = w->bw;
  SeedIn in{};
  in.g_depth = g_depth;
  in.hit_mode = 1;
  launch_samples(w->pool, w->imgs, w->img_order, w->img_latent, n_img, hw, n_lat, tile, in, b->bsum, b->boff,
                 b->seg_base, b->seg_total, b->seg_padded, b->n_samples, b->samples, b->sample_lat, st, 0, nullptr,
                 w->cs->sample_cam);
  AdjArgs aa{};
  aa.net = ctx->net[prec];
  aa.bias0_lat = w->bias0_lat;
  aa.biasS_lat = w->biasS_lat;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  aa.gp_part = w->cs->gp;
  {
    TimedLaunch tl(ctx, 2, st, b->n_samples, 1);
    launch_adjoint(prec, aa, grid, st);
  }
  hipLaunchKernelGGL(k_fill_f32, dim3(512), dim3(256), 0, st, w->cs->gv, npix);
  launch_hit_gv(w->pool, w->imgs, b->samples, w->cs->sample_cam, w->cs->gp, b->n_samples, (int)cap, w->cs->gv, st);
  HIPCHK(hipGetLastError());
  // pass 2: the backward with implicit depth seeds
  return render_bwd(ctx, saved, g_depth, g_normal, g_sil, g_z, nullptr, nullptr, w->cs->gv, st);
}

extern "C" int dist_render_bwd_camera(dist_ctx* ctx, const dist_saved* saved, const float* g_depth,
                                      const float* g_sil, float* g_cam, void* stream) {
  if (!ctx || !saved || !g_cam) return dist_set_error(DIST_EINVAL, "null argument");
  if (saved->ctx != ctx) return dist_set_error(DIST_EINVAL, "saved state belongs to another context");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = saved->ws;
  const int prec = adj_prec(saved->prm.precision);
  const int tile = adj_tile_rows(prec);
  const int n_img = saved->n_img, hw = saved->hw, n_lat = saved->n_lat;
  const long long cap = (long long)n_img * hw * saved->prm.k_samples + (long long)n_lat * tile;
  if (cap > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many gradient samples");
  const int bpi = (hw + 255) / 256;
  const int grid = mlp_grid(ctx, cap, prec);
  int rc = bw_get(ctx, w, (int)cap, n_img * bpi, n_lat, tile, adj_mask_words(prec, ctx->net[prec]) * grid);
  if (!rc) rc = cs_get(ctx, w, cap);
  if (rc) return rc;
  BwdSpace* b = w->bw;
  SeedIn in{};
  in.g_depth = g_depth;
  in.g_sil = g_sil;
  in.nraw = w->nraw;
  in.delta = saved->prm.normal_delta;
  launch_samples(w->pool, w->imgs, w->img_order, w->img_latent, n_img, hw, n_lat, tile, in, b->bsum, b->boff,
                 b->seg_base, b->seg_total, b->seg_padded, b->n_samples, b->samples, b->sample_lat, st, 0, nullptr,
                 w->cs->sample_cam);
  AdjArgs aa{};
  aa.net = ctx->net[prec];
  aa.bias0_lat = w->bias0_lat;
  aa.biasS_lat = w->biasS_lat;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  aa.gp_part = w->cs->gp;
  {
    TimedLaunch tl(ctx, 2, st, b->n_samples, 1);
    launch_adjoint(prec, aa, grid, st);
  }
  launch_cam_reduce(w->pool, w->imgs, w->img_view, n_img, saved->n_views, b->samples, w->cs->sample_cam, w->cs->gp,
                    b->n_samples, g_sil, g_cam, st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

extern "C" int dist_render_bwd_unrolled(dist_ctx* ctx, const dist_saved* saved, const float* g_depth,
                                        const float* g_sil, float* g_z, void* stream) {
  if (!ctx || !saved || !g_z) return dist_set_error(DIST_EINVAL, "null argument");
  if (saved->ctx != ctx) return dist_set_error(DIST_EINVAL, "saved state belongs to another context");
  if (!saved->hist_kept) return dist_set_error(DIST_EINVAL, "the forward did not keep its march history (keep_history)");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = saved->ws;
  const int prec = adj_prec(saved->prm.precision);
  const int tile = adj_tile_rows(prec);
  const int n_img = saved->n_img, hw = saved->hw, n_lat = saved->n_lat;
  const int Lv = saved->prm.c2f_levels, steps = saved->prm.max_steps;
  // one sample per ray of the step's level at most, padded per latent
  const long long cap = (long long)n_img * hw + (long long)n_lat * tile;
  if (cap > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many gradient samples");
  const int bpi = (hw + 255) / 256;
  const int grid = mlp_grid(ctx, cap, prec);
  int rc = bw_get(ctx, w, (int)cap, n_img * bpi, n_lat, tile, adj_mask_words(prec, ctx->net[prec]) * grid);
  if (!rc) rc = cs_get(ctx, w, cap);
  if (rc) return rc;
  BwdSpace* b = w->bw;
  UnrollSpace* u = w->us;
  const int spi = slots_per_image(hw, Lv);
  hipLaunchKernelGGL(k_fill_f32, dim3(64), dim3(256), 0, st, g_z, (long long)n_lat * ctx->L);
  launch_ul_init(w->pool, w->imgs, n_img, spi, g_depth, u->lam, st);
  AdjArgs aa{};
  aa.net = ctx->net[prec];
  aa.bias0_lat = w->bias0_lat;
  aa.biasS_lat = w->biasS_lat;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  aa.gp_part = w->cs->gp;
  const int w0 = ctx->wpad[0];
  const int ws = ctx->skip >= 0 ? ctx->wpad[ctx->skip] : 0;
  for (int n = steps - 1; n >= 0; --n) {
    const int lv = std::max(Lv - n / 3, 0);
    // the rays of level lv + ... have all been processed: after the split
    // that follows step n, the children's adjoints flow to their parents
    if (n % 3 == 2 && lv > 0) launch_ul_split(w->pool, w->imgs, w->img_order, n_img, hw >> (2 * lv), lv, u->lam, st);
    UlIn in{n, lv, g_depth, g_sil, u->t_hist + (size_t)n * w->pool.cap, u->lam};
    launch_ul_samples(w->pool, w->imgs, w->img_order, w->img_latent, n_img, hw >> (2 * lv), n_lat, tile, in, b->bsum,
                      b->boff, b->seg_base, b->seg_total, b->seg_padded, b->n_samples, b->samples, b->sample_lat,
                      w->cs->sample_cam, st);
    {
      TimedLaunch tl(ctx, 2, st, b->n_samples, 1);
      launch_adjoint(prec, aa, grid, st);
    }
    launch_gz_reduce(b->partial, ctx->kmax, tile, (int)(cap / tile) + 1, b->seg_base, b->seg_padded, n_lat, w0,
                     groups_s0(ctx, adjoint_waves()), ctx->w0z, ws, groups_skip(ctx, adjoint_waves()),
                     ctx->skip >= 0 ? ctx->wsz : nullptr, ctx->L, g_z, st, 0, 1);
    launch_ul_lambda(w->pool, b->samples, w->cs->sample_cam, w->cs->gp, b->n_samples, (int)cap, u->lam, st);
  }
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// colour at the hits of a geometry render
// ---------------------------------------------------------------------------
// Buffers of a colour network's calls, grown on demand (held by the context).
static int col_get(dist_ctx* cctx, int n_lat, long long n_pix) {
  ColorSpace* c = cctx->col;
  if (c && c->cap_lat >= n_lat && c->cap_pix >= n_pix) return DIST_OK;
  const int cap_lat = std::max(n_lat, c ? c->cap_lat : 0);
  const long long cap_pix = std::max(n_pix, c ? c->cap_pix : 0LL);
  BwdSpace* keep_bw = c ? c->bw : nullptr;
  if (c) {
    ctx_free(cctx, c->mem, c->bytes);
    delete c;
    cctx->col = nullptr;
  }
  c = new ColorSpace();
  c->bw = keep_bw;
  c->cap_lat = cap_lat;
  c->cap_pix = cap_pix;
  const int ws = cctx->skip >= 0 ? cctx->wpad[cctx->skip] : 0;
  const size_t b0 = (((size_t)cap_lat * cctx->wpad[0] * 4) + 255) & ~(size_t)255;
  const size_t bs = (((size_t)cap_lat * ws * 4) + 255) & ~(size_t)255;
  const size_t li = (((size_t)cap_pix * 4) + 255) & ~(size_t)255;
  c->cap_seed = cap_pix + (long long)cap_lat * 64;
  const size_t cs = (size_t)c->cap_seed * sizeof(float4);
  c->bytes = b0 + bs + li + 256 + cs;
  int rc = ctx_alloc(cctx, (void**)&c->mem, c->bytes);
  if (rc != DIST_OK) {
    if (keep_bw) {
      ctx_free(cctx, keep_bw->mem, keep_bw->bytes);
      delete keep_bw;
    }
    delete c;
    return rc;
  }
  c->bias0 = (float*)c->mem;
  c->biasS = (float*)(c->mem + b0);
  c->list = (int*)(c->mem + b0 + bs);
  c->count = (int*)(c->mem + b0 + bs + li);
  c->cseed = (float4*)(c->mem + b0 + bs + li + 256);
  cctx->col = c;
  return DIST_OK;
}

static int color_check(dist_ctx* cctx, const dist_saved* geom, const float* zc, int32_t n_latents, int32_t precision) {
  if (!cctx || !geom || !zc) return dist_set_error(DIST_EINVAL, "null argument");
  if (cctx->n_out != 3) return dist_set_error(DIST_EINVAL, "not a colour network (last layer width 3)");
  if (geom->ctx->device != cctx->device) return dist_set_error(DIST_EINVAL, "the two networks live on different devices");
  if (n_latents != geom->n_lat) return dist_set_error(DIST_EINVAL, "one colour code per latent of the render");
  if (precision != DIST_FP32 && precision != DIST_BF16)
    return dist_set_error(DIST_EINVAL, "precision must be DIST_FP32 or DIST_BF16");
  return DIST_OK;
}

static void color_fold(dist_ctx* cctx, const float* zc, int n_lat, hipStream_t st) {
  ColorSpace* c = cctx->col;
  launch_fold_bias(cctx->bf[0], cctx->w0z, zc, n_lat, cctx->L, cctx->out_dims[0], cctx->wpad[0], c->bias0, st);
  if (cctx->skip >= 0)
    launch_fold_bias(cctx->bf[cctx->skip], cctx->wsz, zc, n_lat, cctx->L, cctx->out_dims[cctx->skip],
                     cctx->wpad[cctx->skip], c->biasS, st);
}

extern "C" int dist_render_color(dist_ctx* cctx, const dist_saved* geom, const float* zc, int32_t n_latents,
                                 int32_t precision, float* rgb, void* stream) {
  int rc = color_check(cctx, geom, zc, n_latents, precision);
  if (rc) return rc;
  if (!rgb) return dist_set_error(DIST_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(cctx->col_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = geom->ws;
  const int n_img = geom->n_img, hw = geom->hw;
  const long long npix = (long long)n_img * hw;
  rc = col_get(cctx, n_latents, npix);
  if (rc) return rc;
  ColorSpace* c = cctx->col;
  const int prec = precision == DIST_FP32 ? kPrecF32 : kPrecBF16;
  color_fold(cctx, zc, n_latents, st);
  hipLaunchKernelGGL(k_fill_f32, dim3(512), dim3(256), 0, st, rgb, 3 * npix);
  launch_fill_i32(c->count, 0, 1, st);
  launch_color_hits(w->pool, w->imgs, n_img, hw, c->list, c->count, st);
  ColorArgs ca{};
  ca.net = cctx->net[prec];
  ca.pool = w->pool;
  ca.imgs = w->imgs;
  ca.bias0_lat = c->bias0;
  ca.biasS_lat = c->biasS;
  ca.list = c->list;
  ca.count = c->count;
  ca.rgb = rgb;
  launch_color(prec, ca, mlp_grid(cctx, npix, prec), st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

extern "C" int dist_render_color_bwd(dist_ctx* cctx, const dist_saved* geom, const float* zc, int32_t n_latents,
                                     int32_t precision, const float* g_rgb, float* g_zc, void* stream) {
  int rc = color_check(cctx, geom, zc, n_latents, precision);
  if (rc) return rc;
  if (!g_rgb || !g_zc) return dist_set_error(DIST_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(cctx->col_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = geom->ws;
  const int n_img = geom->n_img, hw = geom->hw;
  const long long npix = (long long)n_img * hw;
  // recompute in split bf16 on the bf16 path (as the signed distance's adjoint)
  const int prec = precision == DIST_FP32 ? kPrecF32 : kPrecSplit;
  const int tile = adj_tile_rows(prec);
  const long long cap = npix + (long long)n_latents * tile;
  if (cap > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many gradient samples");
  rc = col_get(cctx, n_latents, npix);
  if (rc) return rc;
  ColorSpace* c = cctx->col;
  const int grid = mlp_grid(cctx, cap, prec);
  const int bpi = (hw + 255) / 256;
  rc = bw_get_into(cctx, c->bw, (int)cap, n_img * bpi, n_latents, tile,
                   adj_mask_words(prec, cctx->net[prec]) * grid);
  if (rc) return rc;
  BwdSpace* b = c->bw;
  color_fold(cctx, zc, n_latents, st);
  launch_color_samples(w->pool, w->imgs, w->img_order, w->img_latent, n_img, hw, n_latents, tile, g_rgb, b->bsum,
                       b->boff, b->seg_base, b->seg_total, b->seg_padded, b->n_samples, b->samples, c->cseed,
                       b->sample_lat, std::min<long long>(cap, c->cap_seed), st);
  AdjArgs aa{};
  aa.net = cctx->net[prec];
  aa.bias0_lat = c->bias0;
  aa.biasS_lat = c->biasS;
  aa.samples = b->samples;
  aa.sample_lat = b->sample_lat;
  aa.n_samples = b->n_samples;
  aa.mask_ws = b->mask_ws;
  aa.partial = b->partial;
  aa.cseed = c->cseed;
  launch_color_adjoint(prec, aa, grid, st);
  const int w0 = cctx->wpad[0];
  const int ws = cctx->skip >= 0 ? cctx->wpad[cctx->skip] : 0;
  // the colour adjoint runs 4 waves: one row group per column sum
  launch_gz_reduce(b->partial, cctx->kmax, tile, (int)(cap / tile) + 1, b->seg_base, b->seg_padded, n_latents, w0, 1,
                   cctx->w0z, ws, 1, cctx->skip >= 0 ? cctx->wsz : nullptr, cctx->L, g_zc, st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// decoder queries at explicit points
// ---------------------------------------------------------------------------
extern "C" int dist_sdf_eval(dist_ctx* ctx, const float* points, const int32_t* latent_ids, const float* z,
                             int32_t n_latents, int64_t n, int32_t precision, float* f, void* stream) {
  if (!ctx) return dist_set_error(DIST_EINVAL, "null argument");
  if (ctx->n_out != 1) return dist_set_error(DIST_EINVAL, "a colour network has no signed distance");
  if (n == 0) return DIST_OK;                       // nothing is read or written
  if (!points || !latent_ids || !z || !f) return dist_set_error(DIST_EINVAL, "null argument");
  if (n < 0 || n > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "n out of range");
  if (n_latents < 1) return dist_set_error(DIST_EINVAL, "n_latents must be positive");
  if (precision < 0 || precision > 2) return dist_set_error(DIST_EINVAL, "bad precision");
  if (n == 0) return DIST_OK;
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  int rc = ws_get(ctx, 1, 1, 1, n_latents, 1, &w);
  if (rc) return rc;
  rc = fold_biases(ctx, w, z, n_latents, st);
  if (!rc) {
    EvalArgs ea{};
    ea.net = ctx->net[precision];
    ea.bias0_lat = w->bias0_lat;
    ea.biasS_lat = w->biasS_lat;
    ea.mode = 0;
    ea.pts = points;
    ea.lat = latent_ids;
    ea.n = n;
    ea.n_lat = n_latents;
    ea.f_out = f;
    {
      TimedLaunch tl(ctx, 1, st);
      launch_eval(precision, ea, mlp_grid(ctx, n, precision), st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = dist_set_error(DIST_EHIP, "eval launch failed: %s", hipGetErrorString(e));
  }
  ws_put(ctx, w);
  return rc;
}

extern "C" int dist_sdf_eval_noalloc(dist_ctx* ctx, const float* points, const int32_t* latent_ids, const float* z,
                                     int32_t n_latents, int64_t n, int32_t precision, float* f, void* stream) {
  if (!ctx) return dist_set_error(DIST_EINVAL, "null argument");
  if (ctx->n_out != 1) return dist_set_error(DIST_EINVAL, "a colour network has no signed distance");
  if (n == 0) return DIST_OK;                       // nothing is read or written
  if (!points || !latent_ids || !z || !f) return dist_set_error(DIST_EINVAL, "null argument");
  if (n < 0 || n > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "n out of range");
  if (n_latents < 1) return dist_set_error(DIST_EINVAL, "n_latents must be positive");
  if (precision < 0 || precision > 2) return dist_set_error(DIST_EINVAL, "bad precision");
  const size_t per_lat = (size_t)ctx->wpad[0] + (ctx->skip >= 0 ? (size_t)ctx->wpad[ctx->skip] : 0);
  if ((size_t)n_latents * per_lat > kNoAllocScratchFloats)
    return dist_set_error(DIST_EINVAL, "n_latents = %d exceeds the allocation-free scratch (%zu floats: at most %zu "
                          "latents for this decoder)", n_latents, kNoAllocScratchFloats,
                          kNoAllocScratchFloats / per_lat);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != ctx->device)
    return dist_set_error(DIST_EINVAL, "the context's device (%d) must be current (device %d is)", ctx->device, dev);
  float* sp = g_scratch_ptr[dev];
  if (!sp) return dist_set_error(DIST_EHIP, "the scratch of device %d was not set up", dev);
  hipStream_t st = (hipStream_t)stream;
  // the folded biases overwrite their whole range, so nothing needs clearing
  float* b0 = sp;
  float* bS = sp + (size_t)n_latents * ctx->wpad[0];
  launch_fold_bias(ctx->bf[0], ctx->w0z, z, n_latents, ctx->L, ctx->out_dims[0], ctx->wpad[0], b0, st);
  if (ctx->skip >= 0)
    launch_fold_bias(ctx->bf[ctx->skip], ctx->wsz, z, n_latents, ctx->L, ctx->out_dims[ctx->skip],
                     ctx->wpad[ctx->skip], bS, st);
  EvalArgs ea{};
  ea.net = ctx->net[precision];
  ea.bias0_lat = b0;
  ea.biasS_lat = ctx->skip >= 0 ? bS : b0;
  ea.mode = 0;
  ea.pts = points;
  ea.lat = latent_ids;
  ea.n = n;
  ea.n_lat = n_latents;
  ea.f_out = f;
  launch_eval(precision, ea, mlp_grid(ctx, n, precision), st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

extern "C" int dist_sdf_vjp(dist_ctx* ctx, const float* points, const int32_t* latent_ids, const float* seeds,
                            const float* z, int32_t n_latents, int64_t n, int32_t precision, float* g_z,
                            float* const* g_W, float* const* g_b, void* stream) {
  if (!ctx || !z || !g_z) return dist_set_error(DIST_EINVAL, "null argument");
  if (ctx->n_out != 1) return dist_set_error(DIST_EINVAL, "a colour network has no signed distance");
  if (n > 0 && (!points || !latent_ids || !seeds)) return dist_set_error(DIST_EINVAL, "null argument");
  if (n < 0 || n > (1LL << 28)) return dist_set_error(DIST_EINVAL, "n out of range");
  if (n_latents < 1) return dist_set_error(DIST_EINVAL, "n_latents must be positive");
  if (precision < 0 || precision > 2) return dist_set_error(DIST_EINVAL, "bad precision");
  if ((g_W == nullptr) != (g_b == nullptr)) return dist_set_error(DIST_EINVAL, "pass both g_W and g_b, or neither");
  precision = adj_prec(precision);
  hipStream_t st = (hipStream_t)stream;
  const int tile = adj_tile_rows(precision);
  // per-latent segments padded to whole tiles: at most n + n_latents (tile - 1) slots
  const long long cap = n + (long long)n_latents * (tile - 1);
  if (cap > (1LL << 31) - 1) return dist_set_error(DIST_EINVAL, "too many samples and latents");
  Workspace* w = nullptr;
  int rc = ws_get(ctx, 1, 1, 1, n_latents, 1, &w);
  if (rc) return rc;
  const int grid = mlp_grid(ctx, std::max<long long>(cap, 1), precision);
  rc = bw_get(ctx, w, (int)std::max<long long>(cap, tile), 1, n_latents, tile,
              adj_mask_words(precision, ctx->net[precision]) * grid);
  if (!rc) rc = gs_get(ctx, w, (int)n, n_latents);
  if (rc) { ws_put(ctx, w); return rc; }
  BwdSpace* b = w->bw;
  GroupSpace* gsp = w->gs;
  rc = fold_biases(ctx, w, z, n_latents, st);
  if (!rc) {
    GroupArgs ga{};
    ga.pts = points;
    ga.seeds = seeds;
    ga.lat = latent_ids;
    ga.n = (int)n;
    ga.n_lat = n_latents;
    ga.tile = tile;
    ga.keys_in = gsp->keys_in;
    ga.vals_in = gsp->vals_in;
    ga.keys_out = gsp->keys_out;
    ga.vals_out = gsp->vals_out;
    ga.cnt = gsp->cnt;
    ga.start = gsp->start;
    ga.temp = gsp->temp;
    ga.temp_bytes = gsp->temp_bytes;
    ga.samples = b->samples;
    ga.sample_lat = b->sample_lat;
    ga.seg_base = b->seg_base;
    ga.seg_total = b->seg_total;
    ga.seg_padded = b->seg_padded;
    ga.n_samples = b->n_samples;
    hipError_t e = group_samples(ga, st);
    if (e != hipSuccess) rc = dist_set_error(DIST_EHIP, "grouping the samples by latent failed: %s", hipGetErrorString(e));
  }
  if (!rc) {
    if (g_W) {
      rc = run_theta(ctx, w, b, precision, z, g_W, g_b, st);
      if (!rc) rc = reduce_only(ctx, b, n_latents, g_z, st);
    } else {
      rc = run_adjoint_and_reduce(ctx, w, b, precision, n_latents, g_z, false, st);
    }
  }
  ws_put(ctx, w);
  return rc;
}

// ---------------------------------------------------------------------------
// image-space loss of inverse optimisation and the optimiser step
// ---------------------------------------------------------------------------
extern "C" int dist_render_loss(int32_t n_images, int32_t H, int32_t W, const float* depth, const float* normal,
                                const float* sil, const float* depth_t, const float* normal_t, const float* sil_t,
                                float w_depth, float w_sil, float w_normal, float* loss, float* g_depth,
                                float* g_normal, float* g_sil, void* stream) {
  if (n_images < 1 || n_images > kMaxImages) return dist_set_error(DIST_EINVAL, "n_images must be in [1, %d]", kMaxImages);
  if (H < 1 || W < 1 || (long long)H * W > (1 << 22))
    return dist_set_error(DIST_EINVAL, "H and W must be positive (at most 4M pixels per image)");
  if (!depth || !sil || !depth_t || !sil_t || !loss) return dist_set_error(DIST_EINVAL, "null argument");
  if (!std::isfinite(w_depth) || !std::isfinite(w_sil) || !std::isfinite(w_normal))
    return dist_set_error(DIST_EINVAL, "loss weights must be finite");
  if (w_normal != 0.f && (!normal || !normal_t))
    return dist_set_error(DIST_EINVAL, "a normal term needs the rendered and the target normals");
  hipStream_t st = (hipStream_t)stream;
  launch_render_loss(depth, normal, sil, depth_t, normal_t, sil_t, n_images, H * W, w_depth, w_sil, w_normal, loss,
                     g_depth, g_normal, g_sil, st);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

extern "C" int dist_adam_step(float* z, float* m, float* v, const float* g, int32_t n, float lr, float beta1,
                              float beta2, float eps, int32_t t, void* stream) {
  if (!z || !m || !v || !g) return dist_set_error(DIST_EINVAL, "null argument");
  if (n < 1) return dist_set_error(DIST_EINVAL, "n must be positive");
  if (t < 1) return dist_set_error(DIST_EINVAL, "the step count t starts at 1");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return dist_set_error(DIST_EINVAL, "need lr > 0, 0 <= beta1, beta2 < 1 and eps > 0");
  launch_adam(z, m, v, g, n, lr, beta1, beta2, eps, t, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return DIST_OK;
}

// ---------------------------------------------------------------------------
// convergence threshold from the camera (host arithmetic only)
// ---------------------------------------------------------------------------
extern "C" int dist_eps_for_camera(double d_min, double sensor, double focal, int32_t resolution, double theta,
                                   double* eps) {
  if (!eps) return dist_set_error(DIST_EINVAL, "null argument");
  if (!(d_min > 0.0) || !(sensor > 0.0) || !(focal > 0.0) || resolution < 1 || !std::isfinite(theta))
    return dist_set_error(DIST_EINVAL, "need d_min, sensor, focal > 0, resolution >= 1 and a finite theta");
  // neighbouring pixels' rays are S / R apart on the sensor; at distance
  // d_min (along the optical axis, the ray tilted by theta) their front ends
  // are d_min (S / R) cos(theta) / (f / cos(theta)) apart, and eps is half of
  // that, so that the eps-balls around them just touch
  const double pitch = sensor / (double)resolution;
  const double c = std::cos(theta);
  *eps = 0.5 * d_min * (pitch * c) / (focal / c);
  return DIST_OK;
}
