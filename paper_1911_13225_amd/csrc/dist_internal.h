// Internal data structures of the MI355X sphere tracer (host + device).
//
// Memory layout in HBM
//   * Ray pool (structure of arrays, one slot per ray of every coarse-to-fine
//     level of every image):  d = (dir.xyz, t) float4, b = (t_lo, t_hi)
//     float2, img int32, st/n uint8 (status, next global step), flast float,
//     and K records of the smallest-|f| queries (rec_f signed f, rec_t, rec_n)
//     stored record-major [K][cap].  An image owns slots
//     [slot_base, slot_base + H*W*(1 + 1/4 + 1/16)): level 0 first, then the
//     coarser levels.
//   * Packed decoder: every hidden-layer weight matrix is stored as MFMA
//     A-operand fragments, fragment-major, so that one wave's fragment is one
//     contiguous 1 KB block (coalesced 16-byte loads, L2 resident).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dist {

constexpr int kMaxLayers = 12;
constexpr int kMaxK = 4;
constexpr int kMaxWidth = 512;

enum : uint8_t { ST_ACTIVE = 0, ST_HIT = 1, ST_MISS = 2, ST_ESCAPED = 3, ST_UNCONVERGED = 4, ST_ERROR = 5 };

// One rendered image: camera, latent, tracing parameters and ray-slot bases.
struct ImgDesc {
  float fx, fy, cx, cy;
  float R[9];                 // camera-to-world rotation, row-major
  float c[3];                 // camera centre
  float alpha, eps, near_, far_;
  int H, W, levels, latent;
  int max_steps, K, cur_level, slot_base;
  int lvl_off[3];             // slot offset of level 0, 1, 2 from slot_base
  int out_base;               // first output pixel of this image
};

struct RayPool {
  float4* d;
  float2* b;
  int* img;
  uint8_t* st;
  uint8_t* n;
  float* flast;
  float* rec_f;
  float* rec_t;
  uint8_t* rec_n;
  int cap;
};

// Device view of a packed decoder for one precision.
struct NetDev {
  int nl, L, skip;                 // layers, latent width, skip layer (-1: none)
  int kmax;                        // widest padded activation row
  int wpad[kMaxLayers];            // padded output width of layers 0 .. nl-2
  int kpad[kMaxLayers];            // padded hidden-part input width of layers 1 .. nl-2
  const void* wp[kMaxLayers];      // W_l packed as A fragments (rows = outputs)
  const void* wpT[kMaxLayers];     // W_l^T packed as A fragments (rows = inputs)
  const void* wplo[kMaxLayers];    // split precision: bf16(W_l - bf16(W_l)) fragments
  const float* bias[kMaxLayers];   // padded biases (float32)
  // the biases as MFMA A fragments (column 0 holds b: float32, or b split in
  // three bf16 parts hi + mid + lo in columns 0-2), so that one MFMA against a
  // ones fragment broadcasts b into the accumulators of a tile
  const void* bfrag[kMaxLayers];
  const float* w0p;                // [3][wpad0]: point columns of layer 0
  const float* wsp;                // [3][wpad_skip]: point columns of the skip layer
  const float* wlast;              // [nout][wpad[nl-2]] output-layer weights
  float blast;                     // output-layer bias (output 0)
  int nout;                        // outputs: 1 (signed distance) or 3 (colour)
  float blast_c[3];                // output-layer biases of a colour network
};

// Colour of the hits of a geometry render (k_color): one row per hit ray.
struct ColorArgs {
  NetDev net;                      // the colour network (nout = 3)
  RayPool pool;                    // the geometry render's rays
  const ImgDesc* imgs;
  const float* bias0_lat;          // folded with the colour codes
  const float* biasS_lat;
  const int* list;                 // hit ray slots
  const int* count;
  float* rgb;                      // [pixels][3]
};

// ---- launchers (defined in the .hip files) --------------------------------
struct MarchArgs {
  NetDev net;
  RayPool pool;
  const ImgDesc* imgs;
  const float* bias0_lat;          // [n_lat][wpad0]  b0 + W0_z z
  const float* biasS_lat;          // [n_lat][wpad_skip]
  const int* list;                 // active ray slots
  const int* count;                // number of entries in list
  // k_march_ring: a second run of *count_tail entries stored backwards from
  // list[tail_end - 1], taken after the first (or null)
  const int* count_tail;
  int tail_end;
  unsigned long long* qcount;      // per-image decoder queries (or null)
  int* ecount;                     // per-image count of non-finite queries (or null)
  // rays still ACTIVE after the step are appended here (null: the caller
  // builds the next list itself, e.g. at a coarse-to-fine split)
  int* next_list;
  int* next_count;
  float* t_hist;                   // [max_steps][pool.cap]: t of each ray at each of its steps (or null)
  unsigned long long* rows_done;   // k_march_ring: queries made, added at the end (or null)
  int* claim;                      // k_march_ring: rays of `list` claimed so far (starts at 0)
  int ring_cap;                    // k_march_ring: ring slots per workgroup in next_list
};

struct EvalArgs {
  NetDev net;
  const float* bias0_lat;
  const float* biasS_lat;
  int mode;                        // 0: explicit points, 1: normal stencil of hits
  const float* pts;                // mode 0: [n][3]
  const int* lat;                  // mode 0: [n]
  long long n;                     // mode 0: count
  int n_lat;                       // mode 0: latent ids are clamped to [0, n_lat)
  const int* hits;                 // mode 1: hit ray slots
  const int* hit_count;            // mode 1: device count of hits
  RayPool pool;
  const ImgDesc* imgs;
  float delta;
  float* f_out;
  // mode 1, optional: per stencil sample i = 6 h + j, the ReLU mask bits of
  // every hidden layer ([i][nl-1][kmax/32] words) and 1 - tanh(m)^2, for a
  // backward that skips the recompute of these samples
  unsigned* mask_out;
  float* dtanh_out;
};

struct AdjArgs {
  NetDev net;
  const float* bias0_lat;
  const float* biasS_lat;
  const float4* samples;           // (p.xyz, seed), grouped by latent, padded per latent
  const int* sample_lat;           // latent of each sample
  const int* n_samples;            // device count (multiple of the tile size)
  unsigned* mask_ws;               // per-workgroup ReLU mask scratch
  float* partial;                  // [tile][2][2][kmax] column sums (S0, Sskip) x m-groups
  // weight gradient (optional): tiles [tile_begin, tile_end) write, per row,
  // h_l (post-ReLU) and Delta_l = seed * dm/d(pre-activation of layer l) for
  // every hidden layer, blocked [nl-1][cap_rows / 64][kmax][64], plus the row's
  // seed factor gm, in the capture type (float32 in the float32 kernel,
  // bfloat16 otherwise)
  float* hbuf;
  float* dbuf;
  float* gmbuf;
  int tile_begin, tile_end;
  int cap_rows;                    // rows of the capture chunk (element l kmax cap_rows + (row / 64 kmax + n) 64 + row % 64)
  // VJP from saved masks (k_vjp_saved): samples [n_begin[0], n_samples[0]),
  // each with its stencil index in sample_idx; masks and 1 - tanh^2 as
  // written by the forward's stencil queries
  const int* n_begin;
  const int* sample_idx;
  const unsigned* smask;
  const float* sdtanh;
  // camera gradient (optional): per sample and wave, gm * (W0_p^T delta0 +
  // Wskip_p^T delta_skip) partial sums over that wave's features,
  // [sample][kGpSlots][3] (the spatial gradient of m, weighted by the row's
  // factor; slots beyond a layer's wave count hold zeros)
  float* gp_part;
  // colour network (k_color_adjoint): per sample dL/d(colour), (r, g, b, 0)
  const float4* cseed;
};

// Precision codes of the decoder kernels: 0 float32, 1 bfloat16, 2 split
// bfloat16 (x = hi + lo, products hi*hi + lo*hi + hi*lo, float32 accumulation).
constexpr int kPrecF32 = 0, kPrecBF16 = 1, kPrecSplit = 2;
constexpr int kGpSlots = 8;          // point-gradient partial slots per sample (one per wave)
constexpr int kMaxImages = 65535;    // images per call: one row each of the per-image launch grids (gridDim.y)

// Inputs of the weight gradient that the capture does not hold, per captured
// row, in the capture's blocked layout (kCapBlock rows per block, a block's
// features contiguous): z of its latent (L features), its point (4: x, y, z,
// 0) and a 1 (for the float32 bias column), in the capture type of
// `precision` (float32 for 0, bfloat16 otherwise); rows in [valid, R) are
// zeros, and so are the captured h, Delta and row factor there.  valid and R
// are multiples of kCapBlock.
void launch_theta_rows(int precision, const float4* pts, const int* lat, const float* z, int L, int valid, int R,
                       void* zrows, void* prows, void* ones, float* hbuf, float* dbuf, float* gmbuf, int n_layers,
                       int kmax, hipStream_t s);
// Weight-gradient contraction over rows (k_dw_bf16 / k_dw_f32): for each
// slice sl of K rows (S slices), P[sl][n][k] (+)= sum_r D[n][r] X_k[r] over
// the slice, for n < n_out, k < kcols, with D and the input features X in
// the capture's blocked layout (rows in blocks of kCapBlock, a block's
// features contiguous, capture type).
constexpr int kCapBlock = 64;                                // rows per capture block (a recompute tile)
struct DwX {
  const void* p[4];          // segment bases (feature 0, block 0 of the segment)
  int end[4];                // cumulative feature counts
  int F[4];                  // features per capture block of the segment (its block stride / kCapBlock)
  int nseg;
};
struct DwArgs {
  const void* D;             // Delta, blocked like the capture
  int FD;                    // features per capture block of D
  DwX x;                     // input features in input order
  int R;                     // feature stride in elements
  int n_out, k_in;           // weight shape; column k_in of a partial holds the bias
  int kcols;                 // columns the GEMM computes (k_in, or k_in + 1 with a ones segment)
  int bias;                  // bf16: the first column block also sums the Delta rows into column k_in
  int K, S;                  // rows per slice (a multiple of kDwRows on the bf16 path), slices
  int acc;                   // add to the partials instead of overwriting them
  int ldp;                   // row stride of a partial (k_in + 1)
  float* P;                  // partials [S][n_out][ldp]
};
constexpr int kDwRows = kCapBlock;                           // rows per LDS block (bf16): one capture block
constexpr int kDwLd = kDwRows + 8;                           // LDS elements per staged feature
constexpr size_t kDwLds = (size_t)2 * 2 * 128 * kDwLd * 2;  // two buffers of both 128-feature tiles
void launch_dw(int precision, const DwArgs& a, hipStream_t s);

int mlp_tile_rows(int precision);                 // rays per MLP tile
int adj_tile_rows(int precision);                 // samples per adjoint tile
size_t mlp_smem_bytes(int precision, const NetDev& net);
size_t adj_mask_words(int precision, const NetDev& net);   // per workgroup
hipError_t mlp_setup(int precision, const NetDev& net);    // raise LDS limits

void launch_march(int precision, const MarchArgs& a, int grid, hipStream_t s);
// every remaining step in one launch (rays claimed from list into per-workgroup rings in next_list)
void launch_march_ring(int precision, const MarchArgs& a, int grid, hipStream_t s);
void launch_eval(int precision, const EvalArgs& a, int grid, hipStream_t s);
// recompute-and-VJP: precision kPrecSplit or kPrecF32 (no bf16 variant; other
// values launch nothing); VJP from saved masks: any precision
void launch_adjoint(int precision, const AdjArgs& a, int grid, hipStream_t s);
// A layer of padded output width `width` run by `waves` waves splits its rows
// into this many groups, each writing its own column sums (the count the
// reduction of dL/dz must add): 2 for 8 waves on a 128-wide layer, else 1.
int mlp_row_groups(int waves, int width);
int adjoint_waves();                       // recompute-and-VJP kernel
int vjp_saved_waves(int precision);        // VJP from saved masks
void launch_vjp_saved(int precision, const AdjArgs& a, int grid, hipStream_t s);
// colour network: forward at hits (precision kPrecF32 or kPrecBF16) and
// recompute + VJP with per-sample colour seeds (kPrecF32 or kPrecSplit)
void launch_color(int precision, const ColorArgs& a, int grid, hipStream_t s);
void launch_color_adjoint(int precision, const AdjArgs& a, int grid, hipStream_t s);

// packing / folding
void launch_pack_bias(int precision, const float* bias, int wpad, void* dst, hipStream_t st);
void launch_pack_w(int precision, bool transpose, const float* W, int out, int in_stride, int ncols,
                   int npad, int kpad, void* dst, hipStream_t s);
void launch_fold_bias(const float* b, const float* Wz, const float* z, int n_lat, int L, int nout,
                      int npad, float* dst, hipStream_t s);

// Grouping of n explicit samples (points [n][3], seeds [n], latent ids [n],
// clamped to [0, n_lat)) into per-latent segments padded to whole tiles of
// the recompute-and-VJP kernel, in sample order within a latent (a stable
// radix sort): samples / sample_lat, seg_base / seg_total / seg_padded per
// latent and the padded total n_samples.  Scratch: keys and values (in and
// out, n each), cnt and start (n_lat each) and temp (temp_bytes, at least
// group_temp_bytes(n, n_lat)).  Stream-ordered, no host synchronisation.
struct GroupArgs {
  const float* pts;
  const float* seeds;
  const int32_t* lat;
  int n, n_lat, tile;
  int *keys_in, *vals_in, *keys_out, *vals_out, *cnt, *start;
  void* temp;
  size_t temp_bytes;
  float4* samples;
  int* sample_lat;
  int *seg_base, *seg_total, *seg_padded, *n_samples;
};
size_t group_temp_bytes(int n, int n_lat);
hipError_t group_samples(const GroupArgs& g, hipStream_t s);

}  // namespace dist
