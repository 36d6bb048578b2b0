// Host-side state of a context, its workspaces and saved forward states.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <mutex>
#include <utility>
#include <vector>

#include "dist.h"
#include "dist_internal.h"

namespace dist {
struct Server;
}

// kernel classes of dist_timing_read: march, decoder queries, adjoint with
// recompute, VJP from saved masks, weight-gradient contraction
constexpr int kTimeClasses = 5;

// Buffers of one backward pass (gradient samples and partial sums).
struct BwdSpace {
  char* mem = nullptr;
  size_t bytes = 0;
  int cap_samples = 0, cap_blocks = 0, cap_lat = 0, tile = 0;
  size_t mask_words = 0;
  float4* samples = nullptr;
  int* sample_lat = nullptr;
  float* partial = nullptr;
  int *bsum = nullptr, *boff = nullptr;
  int *seg_base = nullptr, *seg_total = nullptr, *seg_padded = nullptr;
  int* n_samples = nullptr;       // [end of list 1, its length, end of list 2, its length]
  unsigned* mask_ws = nullptr;
  // second list of the split layout (normal-stencil samples, VJP from saved masks)
  int *bsum2 = nullptr, *boff2 = nullptr;
  int *seg2_base = nullptr, *seg2_total = nullptr, *seg2_padded = nullptr;
  int* sample_idx = nullptr;
  float* partial2 = nullptr;       // column sums of the second list's tiles
};

// ReLU masks and 1 - tanh(m)^2 of the forward's normal-stencil queries, kept
// for a backward that skips their recompute.
struct NrmSave {
  char* mem = nullptr;
  size_t bytes = 0;
  long long cap_samples = 0;
  size_t words = 0;              // mask words per sample
  unsigned* mask = nullptr;
  float* dtanh = nullptr;
};

// Buffers of the camera-extrinsic gradient: per sample its image, pixel and
// ray parameter, and the adjoint's per-wave point-gradient partials.
struct CamSpace {
  char* mem = nullptr;
  size_t bytes = 0;
  long long cap_samples = 0, cap_pix = 0;
  int4* sample_cam = nullptr;
  float* gp = nullptr;
  float* gv = nullptr;             // per output pixel: grad f . v at the hit (implicit depth gradient)
};

// Buffers of the gradient through the unrolled march: the ray parameter of
// every ray slot at every step (kept by the forward) and the per-slot adjoint
// of t.
// Scratch of the device-side grouping of explicit samples by latent
// (dist_sdf_vjp): sort keys and values, per-latent counts and starts, and the
// sort's temporary storage.
struct GroupSpace {
  char* mem = nullptr;
  size_t bytes = 0;
  int cap_n = 0, cap_lat = 0;
  size_t temp_bytes = 0;
  int *keys_in = nullptr, *vals_in = nullptr, *keys_out = nullptr, *vals_out = nullptr;
  int *cnt = nullptr, *start = nullptr;
  void* temp = nullptr;
};

struct UnrollSpace {
  char* mem = nullptr;
  size_t bytes = 0;
  long long cap_hist = 0, cap_lam = 0;
  float* t_hist = nullptr;         // [max_steps][pool capacity]
  float* lam = nullptr;            // [pool capacity]
};

// Buffers of one forward render (ray pool, lists, counters, outputs staging).
struct Workspace {
  char* mem = nullptr;
  size_t bytes = 0;
  int cap_rays = 0, cap_pix = 0, cap_img = 0, cap_lat = 0, cap_steps = 0;
  dist::RayPool pool{};
  dist::ImgDesc* imgs = nullptr;
  int* imgs_list = nullptr;
  int* img_order = nullptr;
  int* img_latent = nullptr;
  int* list[2] = {nullptr, nullptr};
  int* counters = nullptr;
  unsigned long long* qcount = nullptr;
  float* bias0_lat = nullptr;
  float* biasS_lat = nullptr;
  int* hits = nullptr;
  float* fv = nullptr;
  float4* nraw = nullptr;
  int* hit_pix = nullptr;
  int* img_view = nullptr;
  NrmSave* ns = nullptr;
  CamSpace* cs = nullptr;
  UnrollSpace* us = nullptr;
  // pinned staging of the per-call descriptors
  dist::ImgDesc* h_imgs = nullptr;
  int* h_ints = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  BwdSpace* bw = nullptr;
  GroupSpace* gs = nullptr;
};

// Buffers of a colour network's calls (folded biases, hit list, backward).
struct ColorSpace {
  char* mem = nullptr;
  size_t bytes = 0;
  int cap_lat = 0;
  long long cap_pix = 0;
  float* bias0 = nullptr;          // [n_lat][wpad0]
  float* biasS = nullptr;          // [n_lat][wpad_skip]
  int* list = nullptr;             // hit ray slots
  int* count = nullptr;
  float4* cseed = nullptr;         // backward: per sample dL/d(colour)
  long long cap_seed = 0;
  BwdSpace* bw = nullptr;
};

// Capture of one chunk of weight-gradient rows (see run_theta): h and Delta
// of every hidden layer, the row factor, z / point / 1 per row, in the
// blocked layout of the capture (see mlp_kernels.hip) and the capture type of
// the adjoint precision; the slice partials of the contraction, accumulated
// across chunks.
struct ThetaSpace {
  void* mem = nullptr;
  size_t bytes = 0;
  int rows = 0, prec = -1;
  float *hbuf = nullptr, *dbuf = nullptr, *gmbuf = nullptr;
  void *zrows = nullptr, *prows = nullptr, *ones = nullptr;
  float* slices = nullptr;                 // per-slice GEMM results [slice][out][in]
};

struct dist_ctx {
  int device = 0;
  int n_out = 1;                    // 1: signed distance network, 3: colour network
  ColorSpace* col = nullptr;
  std::mutex col_mu;
  int n_cu = 256;
  int nl = 0, L = 0, skip = -1, kmax = 0;
  std::vector<int> out_dims, in_dims, wpad, kpad;
  size_t budget = 0, used = 0;
  std::mutex mem_mu;
  std::vector<std::pair<void*, size_t>> owned;
  std::vector<float*> Wf, bf;            // float32 master copies [out][in], [out]
  std::vector<float*> bias_pad;          // padded hidden biases
  float* w0p = nullptr;                  // [3][wpad0]
  float* w0z = nullptr;                  // [wpad0][L]
  float* wsp = nullptr;                  // [3][wpad_skip]
  float* wsz = nullptr;                  // [wpad_skip][L]
  float* wlast = nullptr;                // [wpad[nl-2]]
  std::vector<void*> wpack[2], wpackT[2], wpacklo, bfrag[2];
  dist::NetDev net[3];          // float32, bfloat16, split bfloat16
  std::mutex ws_mu;
  std::vector<Workspace*> ws_free;
  dist::Server* server = nullptr;
  std::mutex server_mu;
  // kernel timing (see dist_timing_enable)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[kTimeClasses];
  size_t tev_used[kTimeClasses] = {0, 0, 0, 0};
  unsigned long long* d_rows = nullptr;   // device accumulators of processed rows [kTimeClasses]
  // weight gradient: capture buffers of one chunk of rows (kept for the
  // context's life)
  struct ThetaSpace* theta = nullptr;
};

// Event pair around one launch of kernel class k (no-op unless timing is on).
struct TimedLaunch {
  dist_ctx* ctx;
  int k;
  hipStream_t st;
  hipEvent_t end = nullptr;
  TimedLaunch(dist_ctx* c, int kk, hipStream_t s, const int* rows = nullptr, int mul = 1);
  ~TimedLaunch();
};

struct dist_saved {
  dist_ctx* ctx = nullptr;
  Workspace* ws = nullptr;
  const float* z = nullptr;          // the forward's latent codes (caller-owned)
  int n_img = 0, hw = 0, n_lat = 0, n_views = 0;
  dist_trace_params prm{};
  std::vector<int> img_latent, order;
  bool masks_kept = false;           // the stencil queries kept their ReLU masks
  bool hist_kept = false;            // t of every ray at every step is in ws->us
};

int dist_set_error(int code, const char* fmt, ...);

#define HIPCHK_S(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return dist_set_error(DIST_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)
int ctx_alloc(dist_ctx* ctx, void** p, size_t bytes);
void ctx_free(dist_ctx* ctx, void* p, size_t bytes);
int slots_per_image(int hw, int levels);
int fold_biases(dist_ctx* ctx, Workspace* w, const float* z, int n_lat, hipStream_t st);
int run_trace(dist_ctx* ctx, Workspace* w, int n_img, int hw, const dist_trace_params* prm, hipStream_t st,
              float* t_hist = nullptr);
int run_finalize(dist_ctx* ctx, Workspace* w, int n_img, int hw, const dist_trace_params* prm, float* depth,
                 float* dist, float* normal, float* sil, uint8_t* status, uint8_t* nsteps, hipStream_t st,
                 bool keep_masks = false);
void ws_put(dist_ctx* ctx, Workspace* w);
