// Fused decoder kernels for CDNA4 (gfx950): one workgroup evaluates the whole
// DeepSDF-style MLP (paper App. B.1) for a tile of rays or sample points.
//
// Layout of one tile (M rows = rays, 8 waves):
//   * The activation tile lives in LDS, row-major [M][kmax] (bf16 or f32),
//     each row padded by one 16-byte chunk: consecutive rows then start 4
//     banks apart, so the MFMA operand reads (32 rows, one chunk each) and
//     the epilogue writes are bank-conflict free, and a k-step's operand is a
//     lane's row base plus an immediate offset (no per-step address work).
//   * Hidden layers are computed as D[n][m] = sum_k W[n][k] act[m][k] with the
//     weights as the MFMA A operand (pre-packed fragments streamed from L2)
//     and the activations as the B operand (from LDS).  An accumulator lane
//     then holds 4 consecutive output features of one ray, which the
//     epilogue (bias, ReLU, rounding) writes back as one 8/16-byte chunk.
//   * Layer 0 and the point columns of the skip layer are 3-wide products done
//     in float32 on the vector ALUs; the latent part of both is folded into a
//     per-latent bias once per call (z is constant for an image).
//   * The 1-wide output layer is a float32 dot product reduced across waves
//     in a fixed order, then f = 0.5 (|p| - 0.5) + 0.05 tanh(m).
#include "dist_internal.h"
#include "march_rules.h"

namespace dist {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// M rows per tile (MT = M / 32 row tiles), one workgroup per CU.  Each wave
// streams the weight fragments of its own output columns from L2 through the
// vector memory path, the first unit to saturate, so bf16 takes 128-row tiles
// (one weight fragment feeds 4 MFMAs).  The 4-byte formats need 128 KB of LDS
// for 64 rows.
template <int P> struct Cfg;
template <> struct Cfg<1> {           // bf16 x bf16 -> f32, v_mfma_f32_32x32x16_bf16
  static constexpr int M = 128, MT = 4, ES = 2, EPC = 8;
};
template <> struct Cfg<0> {           // f32 x f32 -> f32, v_mfma_f32_32x32x2_f32
  static constexpr int M = 64, MT = 2, ES = 4, EPC = 4;
};
template <> struct Cfg<2> {           // split bf16: x = hi + lo; hi*hi + lo*hi + hi*lo, f32 accumulation
  static constexpr int M = 64, MT = 2, ES = 4, EPC = 8;   // a row holds interleaved hi/lo 16-byte chunks
};

// Waves per workgroup.  8 waves run two per SIMD (at most 256 registers
// each): every wave covers all rows for 1/8 of the outputs (1/4 of a 128-wide
// layer, in two row groups) and the second wave of a SIMD issues while the
// first waits on memory, a barrier or its epilogue.  4 waves run one per SIMD
// with 512 registers (accumulators in AGPRs).  Measured per kernel: the bf16
// and split forward, the recompute-and-VJP and the bf16 VJP from saved masks
// (which takes the forward's 128-row layout) run 8; the float32 forward, the
// split and float32 VJP from saved masks and the colour backward run 4.
template <int P> constexpr int kFwdWaves = P == 0 ? 4 : 8;
constexpr int kBwdWaves = 4;
constexpr int kAdjWaves = 8;
template <int P> constexpr int kVjpWaves = P == 1 ? 8 : 4;

__host__ __device__ inline int rows_for(int P) { return P == 1 ? Cfg<1>::M : 64; }
__host__ __device__ inline int fwd_threads(int P) { return (P == 0 ? 4 : 8) * 64; }
__host__ __device__ inline size_t smem_bytes_for(int P, int kmax, int nout = 1) {
  const int M = rows_for(P);
  const int ES = P == 1 ? 2 : 4;
  return (size_t)M * (kmax * ES + 16) + (size_t)M * (16 + 4 + 4 + 4 + 4) + (size_t)8 * M * 4 * nout;
}

template <int P> struct Sm {
  char* act;
  float4* pts;
  int* lat;
  int* rid;
  float* fval;
  float* gm;
  float* part;
  int rowb;
  __device__ Sm(char* base, int kmax) {
    constexpr int M = Cfg<P>::M;
    rowb = kmax * Cfg<P>::ES + 16;            // one chunk of padding per row
    act = base;
    size_t off = (size_t)M * rowb;
    pts = (float4*)(base + off); off += (size_t)M * 16;
    lat = (int*)(base + off);    off += (size_t)M * 4;
    rid = (int*)(base + off);    off += (size_t)M * 4;
    fval = (float*)(base + off); off += (size_t)M * 4;
    gm = (float*)(base + off);   off += (size_t)M * 4;
    part = (float*)(base + off);
  }
  __device__ __forceinline__ char* chunk(int m, int ch) const {
    return act + (size_t)m * rowb + (ch << 4);
  }
};

extern __shared__ __attribute__((aligned(16))) char dyn_smem[];

// An opaque copy of a lane-dependent value: addresses derived from it are
// computed where they are used instead of being hoisted out of the layer and
// tile loops (which would keep dozens of them alive across the GEMM).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}


// ReLU mask bits of a tile row: word w of layer l of row m is at
// p[row * rs + l * ls + w], with row = m (per-workgroup scratch) or, with rid,
// the row's sample index kept in s.rid (masks saved per sample; rows with a
// negative index are not stored).
struct MaskRef {
  unsigned* p;
  int rs, ls;
  bool rid;
};

template <int P>
__device__ __forceinline__ int mask_row(const MaskRef& mk, const Sm<P>& s, int m) { return mk.rid ? s.rid[m] : m; }

__device__ __forceinline__ size_t mask_at(const MaskRef& mk, int row, int layer, int w) {
  return (size_t)row * mk.rs + (size_t)layer * mk.ls + w;
}

// ---------------------------------------------------------------------------
// Weight-gradient capture (h and Delta of every row and hidden layer, and the
// row factor): float32 elements in the float32 kernels, bfloat16 in the
// others.  The layout is blocked feature-major: rows go in blocks of
// kCapBlock (a tile of the recompute), and element (row r, layer l, feature
// n) of a chunk of R rows is at l kmax R + ((r / kCapBlock) kmax + n)
// kCapBlock + r % kCapBlock.  A feature's rows of one block are contiguous,
// so the contraction over rows reads 8 consecutive rows of one feature as one
// MFMA operand, and a block holds every feature of its rows in one piece: a
// tile writes its capture as one contiguous region and the contraction
// streams its blocks sequentially.  The capture arrays are typed float;
// offsets are in elements of the capture type.
static_assert(Cfg<0>::M == kCapBlock && Cfg<2>::M == kCapBlock, "a recompute tile is one capture block");
template <int P>
__device__ __forceinline__ float* cap_ptr(float* base, size_t off) {
  if constexpr (P == 0) return base + off;
  else return (float*)((bf16*)base + off);
}
// features n..n+3 of row m, below a base that holds the layer and the tile's first row
template <int P>
__device__ __forceinline__ void cap4(float* base, int m, int n, int R, float a, float b, float c, float d) {
  const size_t o = (size_t)n * R + m;
  if constexpr (P == 0) {
    base[o] = a;
    base[o + R] = b;
    base[o + 2 * (size_t)R] = c;
    base[o + 3 * (size_t)R] = d;
  } else {
    bf16* q = (bf16*)base;
    q[o] = (bf16)a;
    q[o + R] = (bf16)b;
    q[o + 2 * (size_t)R] = (bf16)c;
    q[o + 3 * (size_t)R] = (bf16)d;
  }
}
template <int P>
__device__ __forceinline__ float cap_get(const float* base, size_t off) {
  if constexpr (P == 0) return base[off];
  else return (float)((const bf16*)base)[off];
}
template <int P>
__device__ __forceinline__ void cap_put(float* base, size_t off, float v) {
  if constexpr (P == 0) base[off] = v;
  else ((bf16*)base)[off] = (bf16)v;
}

// Capture of a whole tile from LDS, after the barrier that ends a layer: the
// tile's M rows of the layer's first W features, from one plane of the
// activation tile (split bf16: the hi chunks, or the lo chunks where an
// epilogue put the values to capture; float32: the tile itself, each row
// scaled by gm[row] when given).  A thread gathers 8 rows (bf16) or 4 rows
// (float32) of 4 neighbouring features and writes each feature's run of rows
// as one 16-byte store; consecutive threads take consecutive runs of one
// feature, so a wave writes whole 128-byte lines.
template <int P>
__device__ __forceinline__ void cap_tile(const Sm<P>& s, int plane, float* base, int R, int W, const float* gm) {
  constexpr int M = Cfg<P>::M;
  const int nt = blockDim.x;
  if constexpr (P == 2) {
    constexpr int G = M / 8;
    for (int it = threadIdx.x; it < (W / 4) * G; it += nt) {
      const int a = it % G, n = 4 * (it / G);
      uint2 r[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) r[i] = *(const uint2*)(s.chunk(8 * a + i, 2 * (n >> 3) + plane) + 2 * (n & 7));
      bf16* dst = (bf16*)base + (size_t)n * R + 8 * a;
      auto lo2 = [](unsigned x, unsigned y) { return (x & 0xffffu) | (y << 16); };
      auto hi2 = [](unsigned x, unsigned y) { return (x >> 16) | (y & 0xffff0000u); };
      uint4 o;
      o = make_uint4(lo2(r[0].x, r[1].x), lo2(r[2].x, r[3].x), lo2(r[4].x, r[5].x), lo2(r[6].x, r[7].x));
      *(uint4*)dst = o;
      o = make_uint4(hi2(r[0].x, r[1].x), hi2(r[2].x, r[3].x), hi2(r[4].x, r[5].x), hi2(r[6].x, r[7].x));
      *(uint4*)(dst + (size_t)R) = o;
      o = make_uint4(lo2(r[0].y, r[1].y), lo2(r[2].y, r[3].y), lo2(r[4].y, r[5].y), lo2(r[6].y, r[7].y));
      *(uint4*)(dst + 2 * (size_t)R) = o;
      o = make_uint4(hi2(r[0].y, r[1].y), hi2(r[2].y, r[3].y), hi2(r[4].y, r[5].y), hi2(r[6].y, r[7].y));
      *(uint4*)(dst + 3 * (size_t)R) = o;
    }
  } else if constexpr (P == 0) {
    constexpr int G = M / 4;
    for (int it = threadIdx.x; it < (W / 4) * G; it += nt) {
      const int a = it % G, c = it / G;
      float4 r[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        r[i] = *(const float4*)s.chunk(4 * a + i, c);
        if (gm) {
          const float w = gm[4 * a + i];
          r[i] = make_float4(w * r[i].x, w * r[i].y, w * r[i].z, w * r[i].w);
        }
      }
      float* dst = base + (size_t)(4 * c) * R + 4 * a;
      *(float4*)dst = make_float4(r[0].x, r[1].x, r[2].x, r[3].x);
      *(float4*)(dst + (size_t)R) = make_float4(r[0].y, r[1].y, r[2].y, r[3].y);
      *(float4*)(dst + 2 * (size_t)R) = make_float4(r[0].z, r[1].z, r[2].z, r[3].z);
      *(float4*)(dst + 3 * (size_t)R) = make_float4(r[0].w, r[1].w, r[2].w, r[3].w);
    }
  }
}

// ---------------------------------------------------------------------------
// Layer 0: h0 = relu(W0_p p + (b0 + W0_z z)), float32 VALU, written to LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 ld4(const float* p) { return *(const float4*)p; }

// Each thread owns one chunk of EPC output features (its W0_p columns stay in
// registers) and walks the rows of the tile; N0 / EPC divides NT.
// With MASK the ReLU bits of layer 0 are stored like those of the other
// layers (a word holds 32 features, i.e. 32 / EPC neighbouring lanes' chunks,
// combined across those lanes), so the backward reads them instead of
// recomputing W0_p p + b0.
template <int P, int NT, int MR, bool MASK = false>
__device__ __forceinline__ void layer0_fill(const NetDev& net, const float* bias0_lat, const Sm<P>& s, int tid_,
                                            const MaskRef& mk = MaskRef{}) {
  const int tid = opaque(tid_);
  constexpr int M = MR, EPC = Cfg<P>::EPC;
  const int N0 = net.wpad[0];
  const int cpr = N0 / EPC;
  const int rpp = NT / cpr;
  const int ch = tid % cpr;
  const int n = ch * EPC;
  float wx[EPC], wy[EPC], wz[EPC];
#pragma unroll
  for (int e = 0; e < EPC; e += 4) {
    const float4 a = ld4(net.w0p + n + e), b = ld4(net.w0p + N0 + n + e), c = ld4(net.w0p + 2 * N0 + n + e);
    wx[e] = a.x; wx[e + 1] = a.y; wx[e + 2] = a.z; wx[e + 3] = a.w;
    wy[e] = b.x; wy[e + 1] = b.y; wy[e + 2] = b.z; wy[e + 3] = b.w;
    wz[e] = c.x; wz[e + 1] = c.y; wz[e + 2] = c.z; wz[e + 3] = c.w;
  }
  for (int m = tid / cpr; m < M; m += rpp) {
    const float4 p = s.pts[m];
    const float* b0l = bias0_lat + (size_t)s.lat[m] * N0 + n;
    float v[EPC];
#pragma unroll
    for (int e = 0; e < EPC; e += 4) {
      const float4 b = ld4(b0l + e);
      const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        v[e + u] = fmaxf(fmaf(wx[e + u], p.x, fmaf(wy[e + u], p.y, fmaf(wz[e + u], p.z, bb[u]))), 0.f);
    }
    if constexpr (MASK) {
      // v > 0 exactly when the pre-activation is > 0 (the ReLU keeps it)
      constexpr int CPW = 32 / EPC;            // chunks per mask word
      unsigned bits = 0;
#pragma unroll
      for (int e = 0; e < EPC; ++e) bits |= (v[e] > 0.f ? 1u : 0u) << e;
      bits <<= EPC * (ch % CPW);
#pragma unroll
      for (int o = 1; o < CPW; o <<= 1) bits |= __shfl_xor(bits, o);
      const int row = mask_row(mk, s, m);
      if (ch % CPW == 0 && row >= 0) mk.p[mask_at(mk, row, 0, ch / CPW)] = bits;
    }
    if constexpr (P == 1) {
      bf16x8 w;
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = (bf16)v[e];
      *(bf16x8*)s.chunk(m, ch) = w;
    } else if constexpr (P == 2) {
      bf16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hi[e] = (bf16)v[e];
        lo[e] = (bf16)(v[e] - (float)hi[e]);
      }
      *(bf16x8*)s.chunk(m, 2 * ch) = hi;
      *(bf16x8*)s.chunk(m, 2 * ch + 1) = lo;
    } else {
      *(f32x4*)s.chunk(m, ch) = f32x4{v[0], v[1], v[2], v[3]};
    }
  }
}

// ---------------------------------------------------------------------------
// Wave-level GEMM: acc[i][j] (m-tile mt0+i, n-tile nt0+j) += sum_k A[n][k] B[k][m]
// ---------------------------------------------------------------------------
// The k loop is software pipelined: weight fragments (from L2) are requested
// D k-steps before use in a ring of D register sets, and the activation
// fragments of the next k-step (from LDS) are requested one step ahead (a
// double buffer, so the loop is unrolled by U = max(D, 2) steps, an even
// count).  Measured per use: four steps ahead for the bf16 forward (the
// march) and for every VJP (the bf16 one and the split kernels' hi-product
// one: 3-3.5% faster than two), two for the split forward and float32 (1-2%
// either way: fewer loads in flight queue less in the texture units that
// carry them, too few expose the round trip).  The
// last U steps request no weights past the end of the layer.  ksteps must be
// a multiple of U and at least U (the padded widths are multiples of 128).

// Weight fragments are read with raw buffer loads: a scalar resource for the
// layer's packed array (its byte size bounds every load), the lane's 16-byte
// slot as the vector offset and the fragment's position as a scalar offset,
// so stepping k costs no vector address arithmetic.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frag_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
template <class T>
__device__ __forceinline__ T ld_frag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// The epilogue reads the accumulators of the last MFMAs right after the
// GEMM, and a VALU read of a 16-pass MFMA result needs 19 wait states first
// (the CDNA3/4 dependency table).  The compiler's hazard check was seen to
// miss one such read (an integer med3 of the accumulator bits, four
// instructions after the last MFMA), so every GEMM ends with the wait states
// spelled out.
__device__ __forceinline__ void mfma_drain() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <class Frag, int MTW, int NTW, int D>
struct Pipe {
  Frag a[D][NTW];
  Frag b[2][MTW];
};

template <int MTW, int NTW, int D = 2>
__device__ __forceinline__ void gemm_bf16(f32x16 (&acc)[MTW][NTW], const Sm<1>& s, const bf16x8* __restrict__ wp,
                                          int ksteps, int nt0, int mt0, int lane, int nbytes) {
  const int r = lane & 31, g = lane >> 5;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(wp, nbytes);
  const int voff = lane * 16;
  int wrow[NTW];                 // byte offset of fragment (n-tile nt0 + j, k-step 0)
#pragma unroll
  for (int j = 0; j < NTW; ++j) wrow[j] = (nt0 + j) * ksteps * 1024;
  const char* arow[MTW];          // the lane's row and half of the k-step (chunk 2 ks + g)
#pragma unroll
  for (int i = 0; i < MTW; ++i) arow[i] = s.act + (size_t)((mt0 + i) * 32 + r) * s.rowb + 16 * g;
  Pipe<bf16x8, MTW, NTW, D> p;
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < NTW; ++j) p.a[d][j] = ld_frag<bf16x8>(rs, voff, wrow[j] + d * 1024);
    __builtin_amdgcn_sched_barrier(0);     // prologue loads stay in stage order
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) p.b[0][i] = *(const bf16x8*)arow[i];
  constexpr int U = D < 2 ? 2 : D;
  static_assert(U % 2 == 0, "the activation double buffer alternates within a block of U steps");
  // one k-step: the next step's activation fragments (the block's row bases
  // ab plus an immediate; after the layer's last step this reads one chunk
  // past K, still inside the tile, and the value is not used), this step's
  // MFMAs and, with pf, the weight fragments D steps ahead
  const char* ab[MTW];
  auto step = [&](int ks, int d, bool pf) {
    const int sl = d % D, cb = d & 1, nb = cb ^ 1;
#pragma unroll
    for (int i = 0; i < MTW; ++i) p.b[nb][i] = *(const bf16x8*)(ab[i] + 32 * (d + 1));
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int j = 0; j < NTW; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(p.a[sl][j], p.b[cb][i], acc[i][j], 0, 0, 0);
    // the next step's LDS reads spread among this step's MFMAs, one before
    // each group of NTW (left to itself the scheduler sinks them all below
    // the MFMAs and the next step waits for them; measured 2% faster)
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);      // one LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, NTW, 0);    // NTW MFMAs
    }
    if (pf) {
#pragma unroll
      for (int j = 0; j < NTW; ++j) p.a[sl][j] = ld_frag<bf16x8>(rs, voff, wrow[j] + (ks + D) * 1024);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch distance
  };
  // every block but the last prefetches within the layer (ks + D < ksteps);
  // the last block requests no weights past the end
  for (int k0 = 0; k0 < ksteps - U; k0 += U) {
#pragma unroll
    for (int i = 0; i < MTW; ++i) ab[i] = arow[i] + 32 * k0;
#pragma unroll
    for (int d = 0; d < U; ++d) step(k0 + d, d, true);
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) ab[i] = arow[i] + 32 * (ksteps - U);
#pragma unroll
  for (int d = 0; d < U; ++d) step(ksteps - U + d, d, d + D < U);
  mfma_drain();
}

// Split precision: with X3 the product is hi*hi + lo*hi + hi*lo (A = weights,
// B = activations); without X3 only the hi planes are used (bf16 product).
template <int MTW, int NTW, bool X3, int D = 2>
__device__ __forceinline__ void gemm_split(f32x16 (&acc)[MTW][NTW], const Sm<2>& s, const bf16x8* __restrict__ wp,
                                           const bf16x8* __restrict__ wlo, int ksteps, int nt0, int mt0, int lane,
                                           int nbytes) {
  const int r = lane & 31, g = lane >> 5;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(wp, nbytes);
  const __amdgpu_buffer_rsrc_t rl = frag_rsrc(X3 ? wlo : wp, nbytes);
  const int voff = lane * 16;
  int wrow[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) wrow[j] = (nt0 + j) * ksteps * 1024;
  const char* arow[MTW];          // the lane's row and half of the k-step (hi chunk 2 (2 ks + g), lo next)
#pragma unroll
  for (int i = 0; i < MTW; ++i) arow[i] = s.act + (size_t)((mt0 + i) * 32 + r) * s.rowb + 32 * g;
  Pipe<bf16x8, MTW, NTW, D> ph, pl;
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      ph.a[d][j] = ld_frag<bf16x8>(rs, voff, wrow[j] + d * 1024);
      if constexpr (X3) pl.a[d][j] = ld_frag<bf16x8>(rl, voff, wrow[j] + d * 1024);
    }
    __builtin_amdgcn_sched_barrier(0);     // prologue loads stay in stage order
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    ph.b[0][i] = *(const bf16x8*)arow[i];
    if constexpr (X3) pl.b[0][i] = *(const bf16x8*)(arow[i] + 16);
  }
  constexpr int U = D < 2 ? 2 : D;
  static_assert(U % 2 == 0, "the activation double buffer alternates within a block of U steps");
  const char* ab[MTW];           // the block's row bases (see gemm_bf16)
  auto step = [&](int ks, int d, bool pf) {
    const int sl = d % D, cb = d & 1, nb = cb ^ 1;
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      ph.b[nb][i] = *(const bf16x8*)(ab[i] + 64 * (d + 1));
      if constexpr (X3) pl.b[nb][i] = *(const bf16x8*)(ab[i] + 64 * (d + 1) + 16);
    }
    // the next step's LDS reads go out before this step's MFMAs (left to
    // itself the scheduler sinks them below, exposing their latency)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph.a[sl][j], ph.b[cb][i], acc[i][j], 0, 0, 0);
        if constexpr (X3) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl.a[sl][j], ph.b[cb][i], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph.a[sl][j], pl.b[cb][i], acc[i][j], 0, 0, 0);
        }
      }
    if (pf) {
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        ph.a[sl][j] = ld_frag<bf16x8>(rs, voff, wrow[j] + (ks + D) * 1024);
        if constexpr (X3) pl.a[sl][j] = ld_frag<bf16x8>(rl, voff, wrow[j] + (ks + D) * 1024);
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch distance
  };
  for (int k0 = 0; k0 < ksteps - U; k0 += U) {
#pragma unroll
    for (int i = 0; i < MTW; ++i) ab[i] = arow[i] + 64 * k0;
#pragma unroll
    for (int d = 0; d < U; ++d) step(k0 + d, d, true);
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) ab[i] = arow[i] + 64 * (ksteps - U);
#pragma unroll
  for (int d = 0; d < U; ++d) step(ksteps - U + d, d, d + D < U);
  mfma_drain();
}

template <int MTW, int NTW, int D = 2>
__device__ __forceinline__ void gemm_f32(f32x16 (&acc)[MTW][NTW], const Sm<0>& s, const f32x4* __restrict__ wp,
                                         int ksteps, int nt0, int mt0, int lane, int nbytes) {
  const int r = lane & 31, g = lane >> 5;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(wp, nbytes);
  const int voff = lane * 16;
  int wrow[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) wrow[j] = (nt0 + j) * ksteps * 1024;
  const char* arow[MTW];          // the lane's row and half of the k-step (chunk 2 ks + g)
#pragma unroll
  for (int i = 0; i < MTW; ++i) arow[i] = s.act + (size_t)((mt0 + i) * 32 + r) * s.rowb + 16 * g;
  Pipe<f32x4, MTW, NTW, D> p;
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j < NTW; ++j) p.a[d][j] = ld_frag<f32x4>(rs, voff, wrow[j] + d * 1024);
    __builtin_amdgcn_sched_barrier(0);     // prologue loads stay in stage order
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) p.b[0][i] = *(const f32x4*)arow[i];
  constexpr int U = D < 2 ? 2 : D;
  static_assert(U % 2 == 0, "the activation double buffer alternates within a block of U steps");
  for (int k0 = 0; k0 < ksteps; k0 += U) {
    const char* ab[MTW];         // the block's row bases (see gemm_bf16)
#pragma unroll
    for (int i = 0; i < MTW; ++i) ab[i] = arow[i] + 32 * k0;
#pragma unroll
    for (int d = 0; d < U; ++d) {
      const int ks = k0 + d, sl = d % D;
      const int cb = d & 1, nb = cb ^ 1;
#pragma unroll
      for (int i = 0; i < MTW; ++i) p.b[nb][i] = *(const f32x4*)(ab[i] + 32 * (d + 1));
#pragma unroll
      for (int sidx = 0; sidx < 4; ++sidx)
#pragma unroll
        for (int i = 0; i < MTW; ++i)
#pragma unroll
          for (int j = 0; j < NTW; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(p.a[sl][j][sidx], p.b[cb][i][sidx], acc[i][j], 0, 0, 0);
      {
        const int kn = min(ks + D, ksteps - 1);
#pragma unroll
        for (int j = 0; j < NTW; ++j) p.a[sl][j] = ld_frag<f32x4>(rs, voff, wrow[j] + kn * 1024);
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the prefetch distance
    }
  }
  mfma_drain();
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
// EP_VJP_NOGP: the VJP without the point-gradient partials (compiled out)
enum { EP_ACT = 0, EP_LAST = 1, EP_ACT_MASK = 2, EP_LAST_ADJ = 3, EP_VJP = 4, EP_VJP_NOGP = 5 };

struct EpCtx {
  const float* bias;        // per-layer bias (non-skip) or null
  const float* biasS_lat;   // folded skip bias [n_lat][wpad]
  const float* bias0_lat;   // folded layer-0 bias (for the layer-0 mask of the VJP)
  const float* wsp;         // skip point columns [3][wpad]
  int wpad;                 // output width of this layer (stride of biasS/wsp)
  bool skip;                // this layer reads [h, z, p]
  int layer;                // index of the layer whose output this epilogue produces
  MaskRef mk;               // where the ReLU mask bits of each row live
  int ntmax;                // words per mask row of one layer
  float* partial;           // adjoint column-sum output of this tile (or null)
  int which;                // 0: S0, 1: Sskip, -1: none
  bool write_act;
  int kmax;
  float* hrow;              // weight-gradient capture: h of this layer from the tile's first row (or null)
  float* drow;              // weight-gradient capture: Delta of this layer (or null)
  int rstride;              // rows of the capture chunk (feature stride)
  float* gp;                // camera gradient: per-row point-gradient partials [row][kGpSlots][3] (or null)
  int gp_row0;              // global row index of the tile's first row
  bool gp_accum;            // add to the partials (the skip layer wrote them first)
};

// 1 if x > 0, else 0, as an integer clamp med3(bits, 0, 1) of the float's bits
// (no compare, so no lane-mask registers; a NaN with a clear sign bit counts
// as positive).  Written as one instruction: the compiler would turn the
// equivalent min/max back into a compare and a select.
__device__ __forceinline__ unsigned pos_bit(float x) {
  unsigned r;
  asm("v_med3_i32 %0, %1, 0, 1" : "=v"(r) : "v"(x));
  return r;
}

// x if bit b of m is set, else 0 (a bit-field extract and an AND, no compare)
__device__ __forceinline__ float keep_if(float x, unsigned m, int b) {
  return __uint_as_float(__float_as_uint(x) & (0u - ((m >> b) & 1u)));
}

// Lane (r, g) of a wave holds in acc[i][j][4q + e] the output feature
// n = (nt0 + j) * 32 + 8q + 4g + e of tile row m = (mt0 + i) * 32 + r.
__device__ __forceinline__ int feat(int nt0, int j, int q, int g) { return (nt0 + j) * 32 + 8 * q + 4 * g; }

template <int P>
__device__ __forceinline__ void store4(const Sm<P>& s, int m, int n, int g, const float (&v)[4], bool hi_only = false) {
  if constexpr (P == 1) {
    bf16x4 w = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
    *(bf16x4*)(s.chunk(m, n >> 3) + 8 * g) = w;
  } else if constexpr (P == 2) {
    bf16x4 h = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
    *(bf16x4*)(s.chunk(m, 2 * (n >> 3)) + 8 * g) = h;
    if (!hi_only) {
      bf16x4 l = {(bf16)(v[0] - (float)h[0]), (bf16)(v[1] - (float)h[1]), (bf16)(v[2] - (float)h[2]),
                  (bf16)(v[3] - (float)h[3])};
      *(bf16x4*)(s.chunk(m, 2 * (n >> 3) + 1) + 8 * g) = l;
    }
  } else {
    *(f32x4*)s.chunk(m, n >> 2) = f32x4{v[0], v[1], v[2], v[3]};
  }
}

// relu(x) rounded to the tile's activation format and written to LDS.  For
// bf16, rounding first and clearing negative codes (a signed 16-bit max with 0)
// gives the same bits as rounding relu(x).
template <int P>
__device__ __forceinline__ void store4_relu(const Sm<P>& s, int m, int n, int g, const float (&x)[4]) {
  if constexpr (P == 1) {
    typedef short s16x4 __attribute__((ext_vector_type(4)));
    const bf16x4 w = {(bf16)x[0], (bf16)x[1], (bf16)x[2], (bf16)x[3]};
    const s16x4 c = __builtin_elementwise_max(__builtin_bit_cast(s16x4, w), (s16x4)0);
    *(s16x4*)(s.chunk(m, n >> 3) + 8 * g) = c;
  } else {
    const float v[4] = {fmaxf(x[0], 0.f), fmaxf(x[1], 0.f), fmaxf(x[2], 0.f), fmaxf(x[3], 0.f)};
    store4<P>(s, m, n, g, v);
  }
}

template <int MTW, int NTW>
__device__ __forceinline__ void acc_zero(f32x16 (&acc)[MTW][NTW]) {
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
}

// Accumulator start by MFMA: D = A B with A = the bias fragment of the layer
// (column 0: b in float32, or columns 0-2: b = hi + mid + lo in bf16) and B
// a ones fragment (rows 0-2 of every column), C = 0; one MFMA per 32x32 tile
// instead of 16 accumulator writes per lane (the VJP starts from A = 0).
template <int P, int MTW, int NTW>
__device__ __forceinline__ void acc_mfma_start(f32x16 (&acc)[MTW][NTW], const void* bfrag, int nt0, int lane) {
  const int g = lane >> 5;
  const f32x16 zero = {};
  if constexpr (P == 0) {
    const float ones = g == 0 ? 1.f : 0.f;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const float a = bfrag ? ((const float*)bfrag)[(size_t)(nt0 + j) * 64 + lane] : 0.f;
#pragma unroll
      for (int i = 0; i < MTW; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, ones, zero, 0, 0, 0);
    }
  } else {
    const bf16 one = (bf16)(g == 0 ? 1.f : 0.f), z0 = (bf16)0.f;
    const bf16x8 ones = {one, one, one, z0, z0, z0, z0, z0};
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const bf16x8 a = bfrag ? ((const bf16x8*)bfrag)[(size_t)(nt0 + j) * 64 + lane] : bf16x8{};
#pragma unroll
      for (int i = 0; i < MTW; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ones, zero, 0, 0, 0);
    }
  }
}

// Forward layers start the accumulation from the bias, so the epilogue only
// applies the ReLU.  The skip layer's bias is the per-latent folded bias plus
// the float32 point columns W_p p of the row.
template <int P, int MTW, int NTW, bool SKIP>
__device__ __forceinline__ void acc_bias(f32x16 (&acc)[MTW][NTW], const EpCtx& ec, const Sm<P>& s, int nt0, int mt0,
                                         int lane) {
  const int r = lane & 31, g = lane >> 5;
  if constexpr (!SKIP) {
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 b = ld4(ec.bias + feat(nt0, j, q, g));
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
          acc[i][j][4 * q] = b.x;
          acc[i][j][4 * q + 1] = b.y;
          acc[i][j][4 * q + 2] = b.z;
          acc[i][j][4 * q + 3] = b.w;
        }
      }
  } else {
    float4 p[MTW];
    const float* bl[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      const int m = (mt0 + i) * 32 + r;
      p[i] = s.pts[m];
      bl[i] = ec.biasS_lat + (size_t)s.lat[m] * ec.wpad;
    }
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = feat(nt0, j, q, g);
        const float4 wx = ld4(ec.wsp + n), wy = ld4(ec.wsp + ec.wpad + n), wz = ld4(ec.wsp + 2 * ec.wpad + n);
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
          const float4 b = ld4(bl[i] + n);
          acc[i][j][4 * q] = fmaf(wx.x, p[i].x, fmaf(wy.x, p[i].y, fmaf(wz.x, p[i].z, b.x)));
          acc[i][j][4 * q + 1] = fmaf(wx.y, p[i].x, fmaf(wy.y, p[i].y, fmaf(wz.y, p[i].z, b.y)));
          acc[i][j][4 * q + 2] = fmaf(wx.z, p[i].x, fmaf(wy.z, p[i].y, fmaf(wz.z, p[i].z, b.z)));
          acc[i][j][4 * q + 3] = fmaf(wx.w, p[i].x, fmaf(wy.w, p[i].y, fmaf(wz.w, p[i].z, b.w)));
        }
      }
  }
}

// Hidden layer output: relu to LDS (+ ReLU mask bits for the adjoint, + a float32
// copy of h for the weight gradient).
template <int P, int MTW, int NTW, bool MASK, bool CAP>
__device__ __forceinline__ void ep_act(const EpCtx& ec, f32x16 (&acc)[MTW][NTW], const Sm<P>& s, int nt0, int mt0,
                                       int lane) {
  const int r = lane & 31, g = lane >> 5;
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int m = (mt0 + i) * 32 + r;
    const int row = MASK ? mask_row(ec.mk, s, m) : 0;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      unsigned bits = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = feat(nt0, j, q, g);
        const float x[4] = {acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
        if constexpr (MASK) {
#pragma unroll
          for (int e = 0; e < 4; ++e) bits |= pos_bit(x[e]) << (8 * q + e);   // the lane's half: << 4g below
        }
        store4_relu<P>(s, m, n, g, x);
      }
      if constexpr (MASK) {
        bits <<= 4 * g;
        bits |= __shfl_xor(bits, 32);
        if (g == 0 && row >= 0) ec.mk.p[mask_at(ec.mk, row, ec.layer, nt0 + j)] = bits;
      }
    }
  }
}

// Last hidden layer: m-partial = sum_n w_last[n] relu(x[n]) per row (reduced
// across the waves in a fixed order by the caller); with ADJ the seed
// d m / d(pre-activation) = w_last [x > 0] is written to LDS.
template <int P, int MR, int MTW, int NTW, bool ADJ, bool CAP, int NOUT>
__device__ __forceinline__ void ep_last(const NetDev& net, const EpCtx& ec, f32x16 (&acc)[MTW][NTW], const Sm<P>& s,
                                        int nt0, int mt0, int nw, int lane) {
  constexpr int M = MR;
  const int r = lane & 31, g = lane >> 5;
  const int wstride = net.wpad[net.nl - 2];
  float sum[NOUT][MTW];
  unsigned bits[MTW][NTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c) sum[c][i] = 0.f;
#pragma unroll
    for (int j = 0; j < NTW; ++j) bits[i][j] = 0u;
  }
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = feat(nt0, j, q, g);
      float wl[NOUT][4];
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        const float4 w4 = ld4(net.wlast + c * wstride + n);
        wl[c][0] = w4.x;
        wl[c][1] = w4.y;
        wl[c][2] = w4.z;
        wl[c][3] = w4.w;
      }
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const int m = (mt0 + i) * 32 + r;
        float h[4], v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x = acc[i][j][4 * q + e];
          h[e] = fmaxf(x, 0.f);
#pragma unroll
          for (int c = 0; c < NOUT; ++c) sum[c][i] = fmaf(wl[c][e], h[e], sum[c][i]);
          const unsigned b = pos_bit(x);
          v[e] = __uint_as_float(__float_as_uint(wl[0][e]) & (0u - b));
          if constexpr (ADJ) bits[i][j] |= b << (8 * q + e);
        }
        // the seed of the output layer (a single output; a colour network
        // builds its seed from the three channels after the forward)
        if constexpr (ADJ && NOUT == 1) store4<P>(s, m, n, g, v, true);
        if constexpr (CAP && P == 2)
          *(bf16x4*)(s.chunk(m, 2 * (n >> 3) + 1) + 8 * g) = bf16x4{(bf16)h[0], (bf16)h[1], (bf16)h[2], (bf16)h[3]};
        if constexpr (CAP && P == 0) cap4<P>(ec.hrow, m, n, ec.rstride, h[0], h[1], h[2], h[3]);
      }
    }
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int m = (mt0 + i) * 32 + r;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      const float t = sum[c][i] + __shfl_xor(sum[c][i], 32);
      if (g == 0) s.part[(c * 8 + nw) * M + m] = t;
    }
    if constexpr (ADJ) {
      const int row = mask_row(ec.mk, s, m);
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        const unsigned bl = bits[i][j] << (4 * g);
        const unsigned b = bl | __shfl_xor(bl, 32);
        if (g == 0 && row >= 0) ec.mk.p[mask_at(ec.mk, row, ec.layer, nt0 + j)] = b;
      }
    }
  }
}

// VJP through one layer: acc = W^T delta for the output of layer ec.layer;
// apply that layer's ReLU mask, as the forward stored it (layer 0 included).
template <int P, int MTW, int NTW, int WN, bool CAP, bool GP>
__device__ __forceinline__ void ep_vjp(const NetDev& net, const EpCtx& ec, f32x16 (&acc)[MTW][NTW], const Sm<P>& s,
                                       int nt0, int mt0, int mg, int nw, int lane, const unsigned (&mb)[MTW][NTW]) {
  const int r = lane & 31, g = lane >> 5;
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int m = (mt0 + i) * 32 + r;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      // the lane's features are bits 8q + 4g + e of the stored word
      const unsigned bits = mb[i][j] >> (4 * g);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][j][4 * q + e] = keep_if(acc[i][j][4 * q + e], bits, 8 * q + e);
      if (ec.write_act || (CAP && P == 0)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float v[4] = {acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
          store4<P>(s, m, feat(nt0, j, q, g), g, v, true);
        }
      }
      if constexpr (CAP && P == 2) {
        const float w = s.gm[m];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int n = feat(nt0, j, q, g);
          *(bf16x4*)(s.chunk(m, 2 * (n >> 3) + 1) + 8 * g) =
              bf16x4{(bf16)(w * acc[i][j][4 * q]), (bf16)(w * acc[i][j][4 * q + 1]), (bf16)(w * acc[i][j][4 * q + 2]),
                     (bf16)(w * acc[i][j][4 * q + 3])};
        }
      }
    }
  }
  if (GP && ec.gp && ec.which >= 0) {
    // point gradient of m through this layer's point columns, per row:
    // sum_n delta[n] W_p[:, n] over the wave's features, times the row factor
    const float* wp = ec.which == 0 ? net.w0p : net.wsp;
    const int ws = ec.which == 0 ? net.wpad[0] : net.wpad[net.skip];
    float gx[MTW], gy[MTW], gz[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) gx[i] = gy[i] = gz[i] = 0.f;
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = feat(nt0, j, q, g);
        const float4 ax = ld4(wp + n), ay = ld4(wp + ws + n), az = ld4(wp + 2 * ws + n);
        const float wx[4] = {ax.x, ax.y, ax.z, ax.w}, wy[4] = {ay.x, ay.y, ay.z, ay.w},
                    wz[4] = {az.x, az.y, az.z, az.w};
#pragma unroll
        for (int i = 0; i < MTW; ++i)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float d = acc[i][j][4 * q + e];
            gx[i] = fmaf(d, wx[e], gx[i]);
            gy[i] = fmaf(d, wy[e], gy[i]);
            gz[i] = fmaf(d, wz[e], gz[i]);
          }
      }
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      const float x = gx[i] + __shfl_xor(gx[i], 32), y = gy[i] + __shfl_xor(gy[i], 32),
                  z = gz[i] + __shfl_xor(gz[i], 32);
      if (g == 0) {
        const int m = (mt0 + i) * 32 + r;
        const float w = s.gm[m];
        float* dst = ec.gp + ((size_t)(ec.gp_row0 + m) * kGpSlots + nw) * 3;
        if (ec.gp_accum) {
          dst[0] += w * x;
          dst[1] += w * y;
          dst[2] += w * z;
        } else {
          dst[0] = w * x;
          dst[1] = w * y;
          dst[2] = w * z;
          // slots of waves this layer does not have start at zero
#pragma unroll
          for (int k = WN; k < kGpSlots; k += WN) {
            dst[3 * k] = 0.f;
            dst[3 * k + 1] = 0.f;
            dst[3 * k + 2] = 0.f;
          }
        }
      }
    }
  }
  if (ec.which >= 0) {
    // column sums over the tile's rows, each row scaled by its seed gm[m]
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      float cs[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) cs[e] = 0.f;
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const float w = s.gm[(mt0 + i) * 32 + r];
#pragma unroll
        for (int e = 0; e < 16; ++e) cs[e] = fmaf(w, acc[i][j][e], cs[e]);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        float x = cs[e];
        x += __shfl_xor(x, 16);
        x += __shfl_xor(x, 8);
        x += __shfl_xor(x, 4);
        x += __shfl_xor(x, 2);
        x += __shfl_xor(x, 1);
        cs[e] = x;
      }
      if (r == 0) {
        float* dst = ec.partial + ((size_t)(ec.which * 2 + mg)) * ec.kmax;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) dst[feat(nt0, j, q, g) + e] = cs[4 * q + e];
      }
    }
  }
}

// Run one layer (accumulator init + GEMM + barrier + epilogue + barrier) for an
// output width N (128, 256 or 512 after padding): WN waves split N into groups
// of NTW 32-wide tiles; the NW / WN wave groups split the rows into MTW tiles.
template <int P, int MR, int MTW, int NTW, int WN, int MODE, bool CAP, bool SKIP, int NOUT = 1>
__device__ __forceinline__ void layer_run(const NetDev& net, const EpCtx& ec, const Sm<P>& s, const void* wp,
                                          const void* wlo, int ksteps, int nbytes) {
  // lane-dependent addressing is recomputed per layer (see opaque()); the wave
  // index is uniform, so weight addresses are a scalar base plus a lane offset
  const int t = opaque((int)threadIdx.x);
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const int nw = wave % WN, mg = wave / WN;
  const int nt0 = nw * NTW, mt0 = mg * MTW;
  f32x16 acc[MTW][NTW];
  // the VJP's ReLU mask words are requested before the GEMM, so their latency
  // (HBM for saved masks) hides behind it (the bf16 layout has no registers to
  // spare: it reads them in the epilogue)
  unsigned mb[MTW][NTW];
  constexpr bool VJP = MODE == EP_VJP || MODE == EP_VJP_NOGP;
  constexpr bool EARLY = P != kPrecBF16;
  auto load_masks = [&]() {
    const int r = lane & 31;
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int j = 0; j < NTW; ++j)
        mb[i][j] = ec.mk.p[mask_at(ec.mk, max(mask_row(ec.mk, s, (mt0 + i) * 32 + r), 0), ec.layer, nt0 + j)];
  };
  if constexpr (VJP && EARLY) load_masks();
  if constexpr (VJP) acc_mfma_start<P, MTW, NTW>(acc, nullptr, nt0, lane);
  else if constexpr (SKIP) acc_bias<P, MTW, NTW, true>(acc, ec, s, nt0, mt0, lane);
  else acc_mfma_start<P, MTW, NTW>(acc, net.bfrag[ec.layer], nt0, lane);
  if constexpr (P == 1) {
    gemm_bf16<MTW, NTW, 4>(acc, s, (const bf16x8*)wp, ksteps, nt0, mt0, lane, nbytes);
  } else if constexpr (P == 2) {
    gemm_split<MTW, NTW, !VJP, VJP ? 4 : 2>(acc, s, (const bf16x8*)wp, (const bf16x8*)wlo, ksteps, nt0, mt0, lane,
                                         nbytes);
  } else {
    gemm_f32<MTW, NTW>(acc, s, (const f32x4*)wp, ksteps, nt0, mt0, lane, nbytes);
  }
  __syncthreads();
  if constexpr (MODE == EP_ACT) ep_act<P, MTW, NTW, false, CAP>(ec, acc, s, nt0, mt0, lane);
  if constexpr (MODE == EP_ACT_MASK) ep_act<P, MTW, NTW, true, CAP>(ec, acc, s, nt0, mt0, lane);
  if constexpr (MODE == EP_LAST) ep_last<P, MR, MTW, NTW, false, CAP, NOUT>(net, ec, acc, s, nt0, mt0, nw, lane);
  if constexpr (MODE == EP_LAST_ADJ) ep_last<P, MR, MTW, NTW, true, CAP, NOUT>(net, ec, acc, s, nt0, mt0, nw, lane);
  if constexpr (VJP) {
    constexpr bool GP = MODE == EP_VJP;
    if constexpr (!EARLY) load_masks();
    ep_vjp<P, MTW, NTW, WN, CAP, GP>(net, ec, acc, s, nt0, mt0, mg, nw, lane, mb);
  }
  __syncthreads();
  if constexpr (CAP) {
    // weight-gradient capture of the layer's output width from the tile; the
    // next layer's epilogue rewrites the tile only after its GEMM's barrier
    constexpr int N = WN * NTW * 32;
    if constexpr (MODE == EP_ACT || MODE == EP_ACT_MASK) cap_tile<P>(s, 0, ec.hrow, ec.rstride, N, nullptr);
    if constexpr ((MODE == EP_LAST || MODE == EP_LAST_ADJ) && P == 2) cap_tile<P>(s, 1, ec.hrow, ec.rstride, N, nullptr);
    if constexpr (VJP) cap_tile<P>(s, P == 2 ? 1 : 0, ec.drow, ec.rstride, N, P == 0 ? s.gm : nullptr);
  }
}

// One layer of output width N and contracted width K; returns the number of
// wave groups that wrote output-layer partial sums.
// SKIP: the layer reads [h, z, p] (its bias is per latent plus W_p p).
template <int P, int NW, int MR, int MODE, bool CAP, bool SKIP = false, int NOUT = 1>
__device__ __forceinline__ int layer(const NetDev& net, const EpCtx& ec, const Sm<P>& s, const void* wp,
                                     const void* wlo, int N, int K) {
  constexpr int MT = MR / 32;
  const int ksteps = K / (P ? 16 : 8);
  const int nbytes = N * K * (P ? 2 : 4);       // the layer's packed fragment array
  static_assert(NW == 4 || NW == 8, "4 or 8 waves");
  if constexpr (NW == 8) {
    if (N == 512) layer_run<P, MR, MT, 2, 8, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
    else if (N == 256) layer_run<P, MR, MT, 1, 8, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
    else {
      layer_run<P, MR, MT / 2, 1, 4, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
      return 4;
    }
    return 8;
  } else {
    if (N == 512) layer_run<P, MR, MT, 4, 4, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
    else if (N == 256) layer_run<P, MR, MT, 2, 4, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
    else layer_run<P, MR, MT, 1, 4, MODE, CAP, SKIP, NOUT>(net, ec, s, wp, wlo, ksteps, nbytes);
    return 4;
  }
}

__device__ __forceinline__ EpCtx fwd_ctx(const NetDev& net, const float* biasS_lat, int l) {
  EpCtx ec{};
  ec.bias = net.bias[l];
  ec.biasS_lat = biasS_lat;
  ec.wsp = net.wsp;
  ec.wpad = net.wpad[l];
  ec.skip = (l == net.skip);
  ec.layer = l;
  ec.which = -1;
  ec.kmax = net.kmax;
  ec.ntmax = net.kmax / 32;
  return ec;
}

// Forward through all hidden layers; leaves the output-layer partial sums in
// s.part and returns the number of partial groups.  ADJ records the ReLU masks
// and the output-layer seed for the adjoint; CAP keeps float32 copies of every
// hidden activation in hcap (the capture from the tile's first row, chunk
// rows capR) for the weight gradient.
template <int P, int NW, int MR, bool ADJ, bool CAP, int NOUT = 1>
__device__ __forceinline__ int mlp_forward(const NetDev& net, const float* bias0_lat, const float* biasS_lat,
                                           const Sm<P>& s, int tid, const MaskRef& mk, float* hcap = nullptr,
                                           int capR = 0) {
  layer0_fill<P, NW * 64, MR, ADJ>(net, bias0_lat, s, tid, mk);
  __syncthreads();
  if constexpr (CAP) cap_tile<P>(s, 0, hcap, kCapBlock, net.wpad[0], nullptr);
  int wn = 4;
  for (int l = 1; l <= net.nl - 2; ++l) {
    EpCtx ec = fwd_ctx(net, biasS_lat, l);
    ec.mk = mk;
    if constexpr (CAP) {
      ec.hrow = cap_ptr<P>(hcap, (size_t)l * net.kmax * capR);
      ec.rstride = kCapBlock;
    }
    // the skip layer is never the last hidden layer (skip <= nl - 3)
    if (l == net.nl - 2)
      wn = layer<P, NW, MR, ADJ ? EP_LAST_ADJ : EP_LAST, CAP, false, NOUT>(net, ec, s, net.wp[l], net.wplo[l], net.wpad[l], net.kpad[l]);
    else if (l == net.skip)
      wn = layer<P, NW, MR, ADJ ? EP_ACT_MASK : EP_ACT, CAP, true>(net, ec, s, net.wp[l], net.wplo[l], net.wpad[l],
                                                           net.kpad[l]);
    else
      wn = layer<P, NW, MR, ADJ ? EP_ACT_MASK : EP_ACT, CAP>(net, ec, s, net.wp[l], net.wplo[l], net.wpad[l], net.kpad[l]);
  }
  return wn;
}

__device__ __forceinline__ float sdf_from_m(float4 p, float m) {
  const float r = sqrtf(fmaf(p.x, p.x, fmaf(p.y, p.y, p.z * p.z)));
  return 0.5f * (r - 0.5f) + 0.05f * tanhf(m);
}

// Append `value` for every thread with flag set; one atomic per workgroup.
// Called by all threads of the workgroup.
template <int NT>
__device__ __forceinline__ void wg_append(bool flag, int value, int* list, int* counter) {
  __shared__ int wcnt[NT / 64];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(flag);
  const int within = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wcnt[w] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < NT / 64; ++i) tot += wcnt[i];
    base = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  int off = base;
  for (int i = 0; i < w; ++i) off += wcnt[i];
  if (flag) list[off + within] = value;
}

// ---------------------------------------------------------------------------
// March step (Alg. 1 with aggressive steps, convergence and escape; Sec. 3.2)
// ---------------------------------------------------------------------------
// Load the rays of one tile: row i < k takes ray slot rid_of(i), the other
// rows of the M-row tile stay idle (rid -1).  With a history buffer the
// ray's t is recorded at its own step (t_hist[n][slot], stride pool.cap).
template <int P, int M, class RidOf>
__device__ __forceinline__ void march_load(const MarchArgs& a, const Sm<P>& s, int k, RidOf rid_of) {
  const int tid = threadIdx.x;
  if (tid < M) {
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    int lt = 0, r = -1;
    if (tid < k) {
      r = rid_of(tid);
      const ImgDesc& im = a.imgs[a.pool.img[r]];
      const float4 d = a.pool.d[r];
      p = make_float4(fmaf(d.w, d.x, im.c[0]), fmaf(d.w, d.y, im.c[1]), fmaf(d.w, d.z, im.c[2]), 0.f);
      lt = im.latent;
      if (a.t_hist) a.t_hist[(size_t)a.pool.n[r] * a.pool.cap + r] = d.w;
    }
    s.pts[tid] = p;
    s.lat[tid] = lt;
    s.rid[tid] = r;
  }
  __syncthreads();
}

// One decoder query per loaded row and the march epilogue: running top-K of
// |f|, convergence (|f| < eps, Eq. 1), the step limit, the aggressive step
// t += alpha f and the unit-sphere escape test.  Returns whether this
// thread's ray is still ACTIVE; the queries are counted per image.
template <int P, int M>
__device__ __forceinline__ bool march_eval(const MarchArgs& a, const Sm<P>& s) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wn = mlp_forward<P, kFwdWaves<P>, M, false, false>(a.net, a.bias0_lat, a.biasS_lat, s, tid, MaskRef{});
  bool still = false;
  if (tid < M && s.rid[tid] >= 0) {
    float m = a.net.blast;
    for (int w = 0; w < wn; ++w) m += s.part[w * M + tid];
    const float4 p = s.pts[tid];
    const float f = sdf_from_m(p, m);
    const int r = s.rid[tid];
    const RayPool& pl = a.pool;
    const ImgDesc& im = a.imgs[pl.img[r]];
    const int n = pl.n[r];
    float* dw = reinterpret_cast<float*>(pl.d) + 4 * (size_t)r + 3;   // t, the ray's distance
    const float t = *dw;
    // running K smallest |f| (ties keep the earlier step)
    const float af = fabsf(f);
    const int Kr = im.K;
    float rec_abs[kMaxK];
    for (int k = 0; k < Kr; ++k) rec_abs[k] = fabsf(pl.rec_f[(size_t)k * pl.cap + r]);
    const int pos = topk_rank(af, rec_abs, Kr);
    for (int k = Kr - 1; k > pos; --k) {
      pl.rec_f[(size_t)k * pl.cap + r] = pl.rec_f[(size_t)(k - 1) * pl.cap + r];
      pl.rec_t[(size_t)k * pl.cap + r] = pl.rec_t[(size_t)(k - 1) * pl.cap + r];
      pl.rec_n[(size_t)k * pl.cap + r] = pl.rec_n[(size_t)(k - 1) * pl.cap + r];
    }
    if (pos < Kr) {
      pl.rec_f[(size_t)pos * pl.cap + r] = f;
      pl.rec_t[(size_t)pos * pl.cap + r] = t;
      pl.rec_n[(size_t)pos * pl.cap + r] = (uint8_t)n;
    }
    pl.flast[r] = f;
    uint8_t st;
    if (!(af == af) || af == INFINITY) {
      st = ST_ERROR;                         // non-finite query: stop the ray, report it
      if (a.ecount) atomicAdd(&a.ecount[pl.img[r]], 1);
    } else if (af < im.eps) {
      st = ST_HIT;
    } else if (n == im.max_steps - 1) {
      st = ST_UNCONVERGED;
    } else {
      const float tn = fmaf(im.alpha, f, t);
      const float2 b = pl.b[r];
      st = (tn > b.y || tn < b.x) ? ST_ESCAPED : ST_ACTIVE;
      *dw = tn;
    }
    pl.st[r] = st;
    pl.n[r] = (uint8_t)(n + 1);
    still = st == ST_ACTIVE;
  }
  if (a.qcount && tid < M) {
    // queries of this tile per image, one atomic per distinct image in a wave
    const int r = s.rid[tid];
    const bool valid = r >= 0;
    const int img = valid ? a.pool.img[r] : -1;
    unsigned long long todo = __ballot(valid);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int li = __shfl(img, leader);
      const unsigned long long same = __ballot(valid && img == li);
      if (lane == leader) atomicAdd(&a.qcount[li], (unsigned long long)__popcll(same));
      todo &= ~same;
    }
  }
  return still;
}

// One march step over the active list: M-row tiles, the survivors appended to
// the next list (compaction fused into the step).
template <int P, int M>
__device__ __forceinline__ void march_tiles(const MarchArgs& a, const Sm<P>& s, int count) {
  const int tid = threadIdx.x;
  for (int tile = blockIdx.x; tile * M < count; tile += gridDim.x) {
    const int k = min(M, count - tile * M);
    march_load<P, M>(a, s, k, [&](int i) { return a.list[tile * M + i]; });
    const bool still = march_eval<P, M>(a, s);
    if (a.next_list) wg_append<kFwdWaves<P> * 64>(still, still ? s.rid[tid] : 0, a.next_list, a.next_count);
    __syncthreads();
  }
}


// The bf16 step takes 64-row tiles when they finish sooner.  A 64-row tile
// streams the same weights for half the rows, so it is bound by the vector
// memory path and costs about 0.77x a 128-row tile: it wins only when every
// workgroup has at most one tile (the converging tail of the march).
template <int P>
__global__ __launch_bounds__(kFwdWaves<P> * 64) __attribute__((amdgpu_waves_per_eu(kFwdWaves<P> / 4, kFwdWaves<P> / 4))) void k_march(MarchArgs a) {
  Sm<P> s(dyn_smem, a.net.kmax);
  const int count = *a.count;
  if constexpr (P == kPrecBF16) {
    const int g = gridDim.x;
    const int r128 = (count + 128 * g - 1) / (128 * g), r64 = (count + 64 * g - 1) / (64 * g);
    if (r64 * 77 < r128 * 100) march_tiles<P, 64>(a, s, count);
    else march_tiles<P, 128>(a, s, count);
  } else {
    march_tiles<P, Cfg<P>::M>(a, s, count);
  }
}

// Offset of this thread among the workgroup's threads with flag set (thread
// order) and their total, without atomics.
template <int NT>
__device__ __forceinline__ int wg_prefix(bool flag, int* total) {
  __shared__ int pcnt[NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(flag);
  if (lane == 0) pcnt[w] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < NT / 64; ++i) {
    const int c = pcnt[i];
    off += i < w ? c : 0;
    tot += c;
  }
  __syncthreads();                     // pcnt is rewritten by the next call
  *total = tot;
  return off + __popcll(bal & ((1ull << lane) - 1ull));
}

// Every remaining step of the march in one launch (after the last
// coarse-to-fine split).  Each ray's trajectory depends on that ray alone, so
// the rays need not advance in lockstep: every workgroup keeps a ring of rays
// in its own region of a spare list (ring_cap slots), marches tiles of up to
// M of them and puts the survivors back at the ring's end.  While it holds
// fewer than 2M live rays it claims more from the input list (one atomic per
// claim of up to 256), so workgroups that draw short rays take more of them
// and the grid stays busy until the input is spent.  Small claims keep the
// last fresh rays spread over many workgroups: with claims of 1024 the
// workgroups that claimed last still marched hundreds of rays after the
// others had run dry (3% of the march).  No step waits for the
// slowest tile of the grid, and tiles stay full until a workgroup has fewer
// than M live rays.  A ring never overflows: claims are capped by its free
// slots and a ray returns only after leaving it.  Every ray stops within
// max_steps queries and a workgroup leaves once a claim returns nothing and
// its ring is empty, so every workgroup leaves the loop.
template <int P>
__global__ __launch_bounds__(kFwdWaves<P> * 64) __attribute__((amdgpu_waves_per_eu(kFwdWaves<P> / 4, kFwdWaves<P> / 4))) void k_march_ring(MarchArgs a) {
  constexpr int M = Cfg<P>::M, NT = kFwdWaves<P> * 64;
  __shared__ int claim_lds[2];
  Sm<P> s(dyn_smem, a.net.kmax);
  const int tid = threadIdx.x;
  const int nh = *a.count, n0 = nh + (a.count_tail ? *a.count_tail : 0), RC = a.ring_cap;
  int* ring = a.next_list + (size_t)blockIdx.x * RC;
  int head = 0, tail = 0, live = 0;
  bool more = true;
  long long rows = 0;
  while (true) {
    if (more && live < 2 * M) {
      if (tid == 0) {
        const int want = min(256, RC - live);
        const int st = atomicAdd(a.claim, want);
        claim_lds[0] = st;
        claim_lds[1] = max(0, min(want, n0 - st));
      }
      __syncthreads();
      const int st = claim_lds[0], got = claim_lds[1];
      for (int i = tid; i < got; i += NT) {
        const int j = st + i;
        ring[(tail + i) % RC] = j < nh ? a.list[j] : a.list[a.tail_end - 1 - (j - nh)];
      }
      tail += got;
      live += got;
      more = got > 0;
      __syncthreads();
    }
    if (live == 0) break;
    const int k = min(M, live);
    auto rid_of = [&](int i) { return ring[(head + i) % RC]; };
    bool still;
    if (P == kPrecBF16 && k <= 64) {
      march_load<P, 64>(a, s, k, rid_of);
      still = march_eval<P, 64>(a, s);
    } else {
      march_load<P, M>(a, s, k, rid_of);
      still = march_eval<P, M>(a, s);
    }
    int tot;
    const int pos = wg_prefix<NT>(still, &tot);
    if (still) ring[(tail + pos) % RC] = s.rid[tid];
    head += k;
    tail += tot;
    live += tot - k;
    rows += k;
    __syncthreads();
  }
  if (tid == 0 && a.rows_done && rows) atomicAdd(a.rows_done, (unsigned long long)rows);
}

// ---------------------------------------------------------------------------
// Plain decoder queries (explicit points, or the 6-point normal stencil)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kFwdWaves<P> * 64) __attribute__((amdgpu_waves_per_eu(kFwdWaves<P> / 4, kFwdWaves<P> / 4))) void k_eval(EvalArgs a) {
  constexpr int M = Cfg<P>::M;
  Sm<P> s(dyn_smem, a.net.kmax);
  const int tid = threadIdx.x;
  const long long count = a.mode == 0 ? a.n : 6ll * (long long)(*a.hit_count);
  // stencil queries may keep their ReLU masks for the backward (the host
  // only asks for it when every stencil index fits an int)
  const bool keep = P != kPrecBF16 && a.mode == 1 && a.mask_out != nullptr;
  const int ntmax = a.net.kmax / 32;
  const MaskRef mk{a.mask_out, (a.net.nl - 1) * ntmax, ntmax, true};
  for (long long tile = blockIdx.x; tile * M < count; tile += gridDim.x) {
    if (tid < M) {
      const long long idx = tile * M + tid;
      float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
      int lt = 0, row = -1;
      if (idx < count) {
        row = (int)min(idx, (long long)INT_MAX);
        if (a.mode == 0) {
          p = make_float4(a.pts[3 * idx], a.pts[3 * idx + 1], a.pts[3 * idx + 2], 0.f);
          lt = min(max(a.lat[idx], 0), a.n_lat - 1);
        } else {
          const int h = (int)(idx / 6), j = (int)(idx - 6ll * h);
          const int r = a.hits[h];
          const ImgDesc& im = a.imgs[a.pool.img[r]];
          const float4 d = a.pool.d[r];
          const float dd = d.w + a.pool.flast[r];          // Eq. 1 ray distance
          float q[3] = {fmaf(dd, d.x, im.c[0]), fmaf(dd, d.y, im.c[1]), fmaf(dd, d.z, im.c[2])};
          const int ax = j >> 1;
          q[ax] = (j & 1) ? q[ax] - a.delta : q[ax] + a.delta;
          p = make_float4(q[0], q[1], q[2], 0.f);
          lt = im.latent;
        }
      }
      s.pts[tid] = p;
      s.lat[tid] = lt;
      s.rid[tid] = row;
    }
    __syncthreads();
    int wn;
    if constexpr (P != kPrecBF16)
      wn = keep ? mlp_forward<P, kFwdWaves<P>, Cfg<P>::M, true, false>(a.net, a.bias0_lat, a.biasS_lat, s, tid, mk)
                : mlp_forward<P, kFwdWaves<P>, Cfg<P>::M, false, false>(a.net, a.bias0_lat, a.biasS_lat, s, tid, MaskRef{});
    else
      wn = mlp_forward<P, kFwdWaves<P>, Cfg<P>::M, false, false>(a.net, a.bias0_lat, a.biasS_lat, s, tid, MaskRef{});
    if (tid < M && s.rid[tid] >= 0) {
      float m = a.net.blast;
      for (int w = 0; w < wn; ++w) m += s.part[w * M + tid];
      a.f_out[tile * M + tid] = sdf_from_m(s.pts[tid], m);
      if (keep) {
        const float th = tanhf(m);
        a.dtanh_out[tile * M + tid] = 1.f - th * th;
      }
    }
    __syncthreads();
  }
}

// VJP through the hidden layers l = nl-2 .. 1 for the rows of a tile whose
// output-layer seed is in LDS (unit-delta chain; every row is weighted by its
// factor s.gm where the column sums are taken).
template <int P, int NW, bool CAP, bool GP = true>
__device__ __forceinline__ void vjp_layers(const AdjArgs& a, const Sm<P>& s, const MaskRef& mk, float* part,
                                           size_t blk0, int rstride, int tile) {
  const NetDev& net = a.net;
  for (int l = net.nl - 2; l >= 1; --l) {
    EpCtx ec{};
    ec.bias0_lat = a.bias0_lat;
    ec.layer = l - 1;
    ec.mk = mk;
    ec.ntmax = net.kmax / 32;
    ec.partial = part;
    ec.kmax = net.kmax;
    ec.which = (l - 1 == 0) ? 0 : ((l - 1 == net.skip) ? 1 : -1);
    ec.write_act = (l - 1 != 0);
    ec.gp = a.gp_part;
    ec.gp_row0 = tile * Cfg<P>::M;
    ec.gp_accum = (l - 1 == 0) && net.skip >= 1;   // the skip layer comes first in this loop
    if constexpr (CAP) {
      ec.drow = cap_ptr<P>(a.dbuf, (size_t)(l - 1) * net.kmax * a.cap_rows + blk0);
      ec.rstride = kCapBlock;
    }
    layer<P, NW, Cfg<P>::M, GP ? EP_VJP : EP_VJP_NOGP, CAP>(net, ec, s, net.wpT[l], nullptr, net.kpad[l], net.wpad[l]);
  }
}

// ---------------------------------------------------------------------------
// Adjoint: recompute the decoder at detached samples and back-propagate the
// per-sample seeds (Eq. 2 first term, recompute of App. B.2).  Each tile holds
// samples of one latent; it writes the column sums of delta at layer 0 (S0)
// and at the skip layer (Sskip); dL/dz = W0_z^T S0 + Wskip_z^T Sskip.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kAdjWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adjoint(AdjArgs a) {
  constexpr int M = Cfg<P>::M;
  Sm<P> s(dyn_smem, a.net.kmax);
  const NetDev& net = a.net;
  const int tid = threadIdx.x;
  const int count = *a.n_samples;
  const int ntmax = net.kmax / 32;
  const MaskRef mk{a.mask_ws + (size_t)blockIdx.x * (size_t)(net.nl) * M * ntmax, ntmax, M * ntmax, false};
  const bool theta = a.hbuf != nullptr;
  const int t_end = theta ? min(a.tile_end, (count + M - 1) / M) : (count + M - 1) / M;
  const int rstride = a.cap_rows;             // capture chunk rows (feature stride)
  for (int tile = (theta ? a.tile_begin : 0) + blockIdx.x; tile < t_end; tile += gridDim.x) {
    const size_t row0 = theta ? (size_t)(tile - a.tile_begin) * M : 0;   // first row in the chunk
    const size_t blk0 = row0 * net.kmax;                                  // the tile's capture block
    float* hcap = theta ? cap_ptr<P>(a.hbuf, blk0) : nullptr;
    if (tid < M) {
      const int idx = tile * M + tid;
      const float4 smp = a.samples[idx];
      s.pts[tid] = make_float4(smp.x, smp.y, smp.z, 0.f);
      s.fval[tid] = smp.w;
      s.lat[tid] = a.sample_lat[idx];
    }
    __syncthreads();
    const int wn = theta ? mlp_forward<P, kAdjWaves, Cfg<P>::M, true, true>(net, a.bias0_lat, a.biasS_lat, s, tid, mk, hcap,
                                                                            rstride)
                         : mlp_forward<P, kAdjWaves, Cfg<P>::M, true, false>(net, a.bias0_lat, a.biasS_lat, s, tid, mk);
    if (tid < M) {
      float m = net.blast;
      for (int w = 0; w < wn; ++w) m += s.part[w * M + tid];
      const float th = tanhf(m);
      s.gm[tid] = s.fval[tid] * 0.05f * (1.f - th * th);
      if (theta) cap_put<P>(a.gmbuf, row0 + tid, s.gm[tid]);
    }
    __syncthreads();
    if (theta) {
      // Delta of the last hidden layer: gm * w_last * [h > 0]
      const int ll = net.nl - 2, W = net.wpad[ll];
      for (int i = tid; i < M * W; i += kAdjWaves * 64) {
        const int n = i / M, m = i - n * M;          // consecutive threads: consecutive rows of a feature
        const size_t o = (size_t)ll * net.kmax * rstride + blk0 + (size_t)n * kCapBlock + m;
        cap_put<P>(a.dbuf, o, cap_get<P>(a.hbuf, o) > 0.f ? s.gm[m] * net.wlast[n] : 0.f);
      }
    }
    float* part = a.partial + (size_t)tile * 4 * net.kmax;
    if (theta) vjp_layers<P, kAdjWaves, true>(a, s, mk, part, blk0, rstride, tile);
    else vjp_layers<P, kAdjWaves, false>(a, s, mk, part, 0, 0, tile);
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the normal-stencil samples from the ReLU masks their forward
// queries kept: same seeds and VJP as k_adjoint, without the recompute.  The
// output-layer seed w_last [h > 0] is rebuilt from the saved bits of the last
// hidden layer, and the forward's 1 - tanh(m)^2 gives the row factor.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kVjpWaves<P> * 64) __attribute__((amdgpu_waves_per_eu(kVjpWaves<P> / 4, kVjpWaves<P> / 4))) void k_vjp_saved(AdjArgs a) {
  constexpr int M = Cfg<P>::M;
  Sm<P> s(dyn_smem, a.net.kmax);
  const NetDev& net = a.net;
  const int tid = threadIdx.x;
  const int t0 = *a.n_begin / M, t1 = *a.n_samples / M;
  const int ntmax = net.kmax / 32;
  const MaskRef mk{const_cast<unsigned*>(a.smask), (net.nl - 1) * ntmax, ntmax, true};
  const int ll = net.nl - 2, q4 = net.wpad[ll] / 4;
  for (int tile = t0 + blockIdx.x; tile < t1; tile += gridDim.x) {
    if (tid < M) {
      const int idx = tile * M + tid;
      const float4 smp = a.samples[idx];
      const int si = a.sample_idx[idx];
      s.pts[tid] = make_float4(smp.x, smp.y, smp.z, 0.f);
      s.lat[tid] = a.sample_lat[idx];
      s.rid[tid] = si;
      s.gm[tid] = smp.w * 0.05f * a.sdtanh[si];
    }
    __syncthreads();
    for (int i = tid; i < M * q4; i += kVjpWaves<P> * 64) {
      const int m = i / q4, n = 4 * (i - m * q4);
      const unsigned word = a.smask[mask_at(mk, s.rid[m], ll, n >> 5)] >> (n & 31);
      const float4 w4 = ld4(net.wlast + n);
      const float v[4] = {(word & 1u) ? w4.x : 0.f, (word & 2u) ? w4.y : 0.f, (word & 4u) ? w4.z : 0.f,
                          (word & 8u) ? w4.w : 0.f};
      store4<P>(s, m, n, (n >> 2) & 1, v, true);
    }
    __syncthreads();
    // no point gradients here (the camera and unrolled passes use k_adjoint)
    vjp_layers<P, kVjpWaves<P>, false, false>(a, s, mk, a.partial + (size_t)tile * 4 * net.kmax, 0, 0, tile);
  }
}

// ---------------------------------------------------------------------------
// Colour network at the hits of a geometry render (Sec. 3.3, colour rendered
// jointly with the SDF; App. C, the texture network): three outputs, each
// channel 0.5 (1 + tanh(m_c)), at the Eq. 1 point of every hit ray.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kFwdWaves<P> * 64) __attribute__((amdgpu_waves_per_eu(kFwdWaves<P> / 4, kFwdWaves<P> / 4))) void k_color(ColorArgs a) {
  constexpr int M = Cfg<P>::M;
  Sm<P> s(dyn_smem, a.net.kmax);
  const int tid = threadIdx.x;
  const int count = *a.count;
  for (int tile = blockIdx.x; tile * M < count; tile += gridDim.x) {
    if (tid < M) {
      const int idx = tile * M + tid;
      float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
      int lt = 0, r = -1;
      if (idx < count) {
        r = a.list[idx];
        const ImgDesc& im = a.imgs[a.pool.img[r]];
        const float4 d = a.pool.d[r];
        const float dd = d.w + a.pool.flast[r];          // Eq. 1 ray distance
        p = make_float4(fmaf(dd, d.x, im.c[0]), fmaf(dd, d.y, im.c[1]), fmaf(dd, d.z, im.c[2]), 0.f);
        lt = im.latent;
      }
      s.pts[tid] = p;
      s.lat[tid] = lt;
      s.rid[tid] = r;
    }
    __syncthreads();
    const int wn = mlp_forward<P, kFwdWaves<P>, M, false, false, 3>(a.net, a.bias0_lat, a.biasS_lat, s, tid,
                                                                      MaskRef{});
    if (tid < M && s.rid[tid] >= 0) {
      const int r = s.rid[tid];
      const ImgDesc& im = a.imgs[a.pool.img[r]];
      const size_t q = (size_t)im.out_base + (size_t)(r - im.slot_base - im.lvl_off[0]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float m = a.net.blast_c[c];
        for (int w = 0; w < wn; ++w) m += s.part[(c * 8 + w) * M + tid];
        a.rgb[3 * q + c] = 0.5f * (1.f + tanhf(m));
      }
    }
    __syncthreads();
  }
}

// Backward of the colour: recompute at the (detached) hit points with masks in
// per-workgroup scratch, seed the last hidden layer with
// sum_c g_c 0.5 (1 - tanh^2 m_c) w_last[c] on its active units, and run the
// VJP with unit row weights; the column sums at layer 0 and the skip layer
// give dL/dz per latent as for the signed distance.
template <int P>
__global__ __launch_bounds__(kBwdWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_color_adjoint(AdjArgs a) {
  constexpr int M = Cfg<P>::M;
  constexpr int NT = kBwdWaves * 64;
  Sm<P> s(dyn_smem, a.net.kmax);
  const NetDev& net = a.net;
  const int tid = threadIdx.x;
  const int count = *a.n_samples;
  const int ntmax = net.kmax / 32;
  const MaskRef mk{a.mask_ws + (size_t)blockIdx.x * (size_t)(net.nl) * M * ntmax, ntmax, M * ntmax, false};
  const int ll = net.nl - 2, W = net.wpad[ll], q4 = W / 4;
  for (int tile = blockIdx.x; tile * M < count; tile += gridDim.x) {
    if (tid < M) {
      const float4 smp = a.samples[tile * M + tid];
      s.pts[tid] = make_float4(smp.x, smp.y, smp.z, 0.f);
      s.lat[tid] = a.sample_lat[tile * M + tid];
    }
    __syncthreads();
    const int wn = mlp_forward<P, kBwdWaves, M, true, false, 3>(net, a.bias0_lat, a.biasS_lat, s, tid, mk);
    if (tid < M) {
      const float4 g = a.cseed[tile * M + tid];
      const float gc[3] = {g.x, g.y, g.z};
      float ac[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float m = net.blast_c[c];
        for (int w = 0; w < wn; ++w) m += s.part[(c * 8 + w) * M + tid];
        const float th = tanhf(m);
        ac[c] = gc[c] * 0.5f * (1.f - th * th);
      }
      // this row's partial-sum slots are read: they now keep its channel factors
#pragma unroll
      for (int c = 0; c < 3; ++c) s.part[c * 8 * M + tid] = ac[c];
      s.gm[tid] = 1.f;
    }
    __syncthreads();
    for (int i = tid; i < M * q4; i += NT) {
      const int m = i / q4, n = 4 * (i - m * q4);
      const unsigned word = mk.p[mask_at(mk, m, ll, n >> 5)] >> (n & 31);
      const float a0 = s.part[m], a1 = s.part[8 * M + m], a2 = s.part[16 * M + m];
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float d = fmaf(a0, net.wlast[n + e], fmaf(a1, net.wlast[W + n + e], a2 * net.wlast[2 * W + n + e]));
        v[e] = ((word >> e) & 1u) ? d : 0.f;
      }
      store4<P>(s, m, n, (n >> 2) & 1, v, true);
    }
    __syncthreads();
    vjp_layers<P, kBwdWaves, false, false>(a, s, mk, a.partial + (size_t)tile * 4 * net.kmax, 0, 0, tile);
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of one layer from captured rows (fixed summation order):
//   gW[n][k] += sum_r Delta_l[r][n] * in_l(r, k),  gb[n] += sum_r Delta_l[r][n]
// in_l is [z, p] for layer 0, [h, z, p] for the skip layer, h_{l-1} otherwise;
// for the output layer Delta is the row's seed factor gm and in = h_{nl-2}.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
int mlp_tile_rows(int precision) { return rows_for(precision); }

int adj_tile_rows(int precision) { return mlp_tile_rows(precision); }
size_t mlp_smem_bytes(int precision, const NetDev& net) { return smem_bytes_for(precision, net.kmax, net.nout); }
size_t adj_mask_words(int precision, const NetDev& net) {
  return (size_t)net.nl * mlp_tile_rows(precision) * (net.kmax / 32);
}

// Per captured row, in the blocked layout of the capture (features of a
// kCapBlock-row block contiguous): z of its latent, its point (and a 0) and a
// 1, in the capture type; for the rows in [valid, R) that only pad the
// contraction to whole slices, zeros there and in the captured h, Delta and
// row factor (whole blocks: valid is a multiple of kCapBlock).
template <class T>
__global__ void k_theta_rows(const float4* __restrict__ pts, const int* __restrict__ lat, const float* __restrict__ z,
                             int L, int valid, int R, T* zrows, T* prows, T* ones, T* hbuf, T* dbuf, T* gmbuf,
                             int n_layers, int kmax) {
  const long long step = (long long)gridDim.x * blockDim.x, t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  constexpr int B = kCapBlock;
  for (long long i = t0; i < (long long)L * R; i += step) {
    // i walks the blocked layout: block b, feature j, row r % B
    const long long b = i / ((long long)L * B);
    const int j = (int)(i / B % L), r = (int)(b * B + i % B);
    zrows[i] = (T)(r < valid ? z[(size_t)lat[r] * L + j] : 0.f);
  }
  for (long long r = t0; r < R; r += step) {
    const bool ok = r < valid;
    const float4 p = ok ? pts[r] : make_float4(0.f, 0.f, 0.f, 0.f);
    T* pr = prows + (r / B) * 4 * B + r % B;
    pr[0] = (T)p.x;
    pr[B] = (T)p.y;
    pr[2 * B] = (T)p.z;
    pr[3 * B] = (T)0.f;
    ones[r] = (T)(ok ? 1.f : 0.f);
    if (!ok) gmbuf[r] = (T)0.f;
  }
  // padding blocks of every layer: one contiguous range per layer
  const long long per = (long long)(R - valid) * kmax;
  for (long long i = t0; i < (long long)n_layers * per; i += step) {
    const long long l = i / per, o = l * kmax * R + (long long)valid * kmax + (i - l * per);
    hbuf[o] = (T)0.f;
    dbuf[o] = (T)0.f;
  }
}

void launch_theta_rows(int precision, const float4* pts, const int* lat, const float* z, int L, int valid, int R,
                       void* zrows, void* prows, void* ones, float* hbuf, float* dbuf, float* gmbuf, int n_layers,
                       int kmax, hipStream_t st) {
  const long long total = (long long)std::max(L, 1) * R;
  const int grid = (int)std::min<long long>((total + 255) / 256, 4096);
  if (precision == 0)
    hipLaunchKernelGGL(k_theta_rows<float>, dim3(grid), dim3(256), 0, st, pts, lat, z, L, valid, R, (float*)zrows,
                       (float*)prows, (float*)ones, hbuf, dbuf, gmbuf, n_layers, kmax);
  else
    hipLaunchKernelGGL(k_theta_rows<bf16>, dim3(grid), dim3(256), 0, st, pts, lat, z, L, valid, R, (bf16*)zrows,
                       (bf16*)prows, (bf16*)ones, (bf16*)hbuf, (bf16*)dbuf, (bf16*)gmbuf, n_layers, kmax);
}

// Weight-gradient contraction over the captured rows (Sec. 3.4: dW_l = sum
// over samples of Delta_l x_l^T, db_l = sum of Delta_l): for each slice sl of
// K rows, P[sl][n][k] = sum over the slice's rows r of D[n][r] X[k][r], with
// D and X in the capture's blocked layout (64-row blocks, a block's features
// contiguous, each segment with its own features per block).  The input features X of a layer
// are up to four segments in input order (h, z, p, and on the float32 path a
// ones row that yields the bias column).  With acc set the slice adds to the
// partial it holds from the previous chunk; every slice is owned by one
// workgroup per launch, so the sum order is fixed.  Slices are mapped to
// workgroups so that all tiles of one slice run on one XCD (workgroups are
// dealt to the 8 XCDs round robin) and share its L2 for the slice's rows.
// input feature k: its rows of block 0 and the block stride (elements)
__device__ __forceinline__ const char* dw_feature(const DwX& x, int k, int es, int& bstride) {
  const void* b = x.p[0];
  int base = 0, F = x.F[0];
  if (x.nseg > 1 && k >= x.end[0]) { b = x.p[1]; base = x.end[0]; F = x.F[1]; }
  if (x.nseg > 2 && k >= x.end[1]) { b = x.p[2]; base = x.end[1]; F = x.F[2]; }
  if (x.nseg > 3 && k >= x.end[2]) { b = x.p[3]; base = x.end[2]; F = x.F[3]; }
  bstride = F * kCapBlock;
  return (const char*)b + (size_t)(k - base) * kCapBlock * es;
}

// workgroup -> (tile of the output, slice), all tiles of a slice on one XCD
__device__ __forceinline__ void dw_block(int T, int S, int& tile, int& slice) {
  const int id = blockIdx.x;
  if (S % 8 == 0) {
    const int x = id & 7, y = id >> 3;
    slice = (y / T) * 8 + x;
    tile = y % T;
  } else {
    slice = id / T;
    tile = id % T;
  }
}

__device__ __forceinline__ void dw_put(const DwArgs& a, float* P, int n, int k, float v) {
  float* d = P + (size_t)n * a.ldp + k;
  *d = a.acc ? *d + v : v;
}

// bf16: a workgroup of 4 waves owns a 128 (n) x 128 (k) block.  Blocks of
// kDwRows rows of both operands are staged in LDS (feature-major, one padded
// row of kDwLd elements per feature) with 16-byte loads, 8 lanes per 128-byte
// feature row, double buffered: the next block's loads are in flight while
// the MFMAs run on the current one.  Each wave computes 64 x 64 as 2 x 2
// 32x32x16 tiles whose A operand is 8 rows of one Delta feature and B
// operand 8 rows of one input feature.  The workgroups of the first k-block
// column also sum the staged Delta rows: the bias column (k_in) of the
// partial.  Features past n_out or kcols are clamped to the last one and
// their outputs dropped.
__global__ __launch_bounds__(256, 2) void k_dw_bf16(DwArgs a) {
  bf16* lds = (bf16*)dyn_smem;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, ln = lane & 31, g = lane >> 5;
  const int Tn = (a.n_out + 127) / 128, Tk = (a.kcols + 127) / 128;
  int tile, slice;
  dw_block(Tn * Tk, a.S, tile, slice);
  const int n0 = (tile % Tn) * 128, k0 = (tile / Tn) * 128;
  const size_t r0 = (size_t)slice * a.K;
  const int rc = t & 7, fl = t >> 3;
  const bf16* ga[4];
  const bf16* gx[4];
  int sx[4];                              // block strides of the input features (segments differ)
  const int sa = a.FD * kCapBlock;
  const size_t b0 = r0 / kCapBlock;       // the slice's first block
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int n = min(n0 + fl + 32 * i, a.n_out - 1), k = min(k0 + fl + 32 * i, a.kcols - 1);
    ga[i] = (const bf16*)a.D + b0 * sa + (size_t)n * kCapBlock + 8 * rc;
    gx[i] = (const bf16*)dw_feature(a.x, k, 2, sx[i]);
    gx[i] += b0 * sx[i] + 8 * rc;
  }
  const bool bias = k0 == 0 && a.bias;
  float bs[4] = {0.f, 0.f, 0.f, 0.f};
  // three register sets: the loads of blocks b + 2 and b + 3 are in flight
  // while block b is multiplied from LDS and block b + 1 is staged (HBM
  // latency under load needs about that many bytes in flight per CU)
  constexpr int NS = 3;
  bf16x8 ra[NS][4], rx[NS][4];
  auto gload = [&](int set, int blk) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ra[set][i] = *(const bf16x8*)(ga[i] + (size_t)blk * sa);
      rx[set][i] = *(const bf16x8*)(gx[i] + (size_t)blk * sx[i]);
    }
  };
  auto stage = [&](int set, int buf) {
    bf16* A = lds + (size_t)buf * 2 * 128 * kDwLd;
    bf16* X = A + 128 * kDwLd;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *(bf16x8*)(A + (fl + 32 * i) * kDwLd + 8 * rc) = ra[set][i];
      *(bf16x8*)(X + (fl + 32 * i) * kDwLd + 8 * rc) = rx[set][i];
    }
    if (bias) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 8; ++e) bs[i] += (float)ra[set][i][e];
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};
  const int wn = wave & 1, wk = wave >> 1;
  const int nblk = a.K / kDwRows;
  auto mma = [&](int buf) {
    const bf16* A = lds + (size_t)buf * 2 * 128 * kDwLd;
    const bf16* X = A + 128 * kDwLd;
#pragma unroll
    for (int ks = 0; ks < kDwRows / 16; ++ks) {
      bf16x8 av[2], xv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = *(const bf16x8*)(A + (64 * wn + 32 * i + ln) * kDwLd + 16 * ks + 8 * g);
        xv[i] = *(const bf16x8*)(X + (64 * wk + 32 * i + ln) * kDwLd + 16 * ks + 8 * g);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], xv[j], acc[i][j], 0, 0, 0);
    }
  };
  // block b sits in register set b % NS, then in LDS buffer b % 2.  The loads
  // are issued unconditionally (past the last block they repeat it, in
  // bounds and unused): a conditional load would make the wait for an older
  // set count it as absent and drain everything in flight.
  auto step = [&](int blk, int set, int buf) {
    gload(set, min(blk + NS, nblk - 1));
    // the loads go out before the MFMAs (left to itself the scheduler sinks
    // them below the wait for the older sets)
    __builtin_amdgcn_sched_barrier(0);
    mma(buf);
    __builtin_amdgcn_sched_barrier(0);
    if (blk + 1 < nblk) stage((set + 1) % NS, buf ^ 1);
    __syncthreads();
  };
#pragma unroll
  for (int u = 0; u < NS; ++u) gload(u, min(u, nblk - 1));
  stage(0, 0);
  __syncthreads();
  int blk = 0;
  for (; blk + 6 <= nblk; blk += 6) {
#pragma unroll
    for (int u = 0; u < 6; ++u) step(blk + u, u % NS, u & 1);
  }
#pragma unroll
  for (int u = 0; u < 6; ++u)                     // the last nblk % 6 blocks (register sets indexed statically)
    if (blk + u < nblk) step(blk + u, u % NS, u & 1);
  mfma_drain();
  float* P = a.P + (size_t)slice * a.n_out * a.ldp;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = n0 + 64 * wn + 32 * i + 8 * q + 4 * g + e, k = k0 + 64 * wk + 32 * j + ln;
          if (n < a.n_out && k < a.kcols) dw_put(a, P, n, k, acc[i][j][4 * q + e]);
        }
  if (bias) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float x = bs[i];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      const int n = n0 + fl + 32 * i;
      if (rc == 0 && n < a.n_out) dw_put(a, P, n, a.k_in, x);
    }
  }
}

// float32: the operands are read straight from memory (float4 of 4 rows per
// lane), a workgroup of 4 waves owns 128 x 128 and a wave 64 x 64 as 2 x 2
// 32x32x2 tiles, the rows paired (i, i + 4) (any pairing of the contraction
// index gives the same sum); the bias comes from the ones segment.
__global__ __launch_bounds__(256) void k_dw_f32(DwArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 31, g = lane >> 5;
  const int Tn = (a.n_out + 127) / 128, Tk = (a.kcols + 127) / 128;
  int tile, slice;
  dw_block(Tn * Tk, a.S, tile, slice);
  const int nb = (tile % Tn) * 128 + (wave & 1) * 64, kb = (tile / Tn) * 128 + (wave >> 1) * 64;
  const size_t r0 = (size_t)slice * a.K;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};
  const float* pa[2];
  const float* pb[2];
  int sb[2];
  const int sa = a.FD * kCapBlock;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    pa[i] = (const float*)a.D + (size_t)min(nb + 32 * i + ln, a.n_out - 1) * kCapBlock + 4 * g;
    pb[i] = (const float*)dw_feature(a.x, min(kb + 32 * i + ln, a.kcols - 1), 4, sb[i]) + 4 * g;
  }
  for (int r = 0; r < a.K; r += 8) {
    const size_t blk = (r0 + r) / kCapBlock, w = (r0 + r) % kCapBlock;
    float4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      av[i] = *(const float4*)(pa[i] + blk * sa + w);
      bv[i] = *(const float4*)(pb[i] + blk * sb[i] + w);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].x, bv[j].x, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].y, bv[j].y, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].z, bv[j].z, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].w, bv[j].w, acc[i][j], 0, 0, 0);
      }
  }
  mfma_drain();
  float* P = a.P + (size_t)slice * a.n_out * a.ldp;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = nb + 32 * i + 8 * q + 4 * g + e, k = kb + 32 * j + ln;
          if (n < a.n_out && k < a.kcols) dw_put(a, P, n, k, acc[i][j][4 * q + e]);
        }
}

void launch_dw(int precision, const DwArgs& a, hipStream_t st) {
  const int T = ((a.n_out + 127) / 128) * ((a.kcols + 127) / 128);
  const dim3 grid(T * a.S);
  if (precision == 0) hipLaunchKernelGGL(k_dw_f32, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_dw_bf16, grid, dim3(256), kDwLds, st, a);
}

template <int P>
static hipError_t setup_p(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_march<P>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_eval<P>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_vjp_saved<P>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess || P == kPrecBF16) return e;          // the recompute has no bf16 kernel
  return hipFuncSetAttribute((const void*)k_adjoint<P == kPrecBF16 ? kPrecSplit : P>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t mlp_setup(int precision, const NetDev& net) {
  const int bytes = (int)mlp_smem_bytes(precision, net);
  if (net.nout == 3) {                     // a colour network: its own kernels only
    if (precision == 1)
      return hipFuncSetAttribute((const void*)k_color<1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (precision == 2)
      return hipFuncSetAttribute((const void*)k_color_adjoint<2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    hipError_t e = hipFuncSetAttribute((const void*)k_color<0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_color_adjoint<0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  }
  if (precision == 1) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dw_bf16, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDwLds);
    if (e != hipSuccess) return e;
    return setup_p<1>(bytes);
  }
  if (precision == 2) return setup_p<2>(bytes);
  return setup_p<0>(bytes);
}

#define DIST_DISPATCH(KERNEL, ARGS)                                                                    \
  do {                                                                                                 \
    const size_t sm = mlp_smem_bytes(precision, ARGS.net);                                             \
    const dim3 blk(fwd_threads(precision));                                                            \
    if (precision == 1) hipLaunchKernelGGL(KERNEL<1>, dim3(grid), blk, sm, st, ARGS);                  \
    else if (precision == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(grid), blk, sm, st, ARGS);             \
    else hipLaunchKernelGGL(KERNEL<0>, dim3(grid), blk, sm, st, ARGS);                                 \
  } while (0)

// the recompute-and-VJP kernel exists in split and float32 precision only
#define DIST_DISPATCH_BWD(KERNEL, ARGS)                                                                \
  do {                                                                                                 \
    const size_t sm = mlp_smem_bytes(precision, ARGS.net);                                             \
    const dim3 blk(kAdjWaves * 64);                                                                    \
    if (precision == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(grid), blk, sm, st, ARGS);                  \
    else if (precision == 0) hipLaunchKernelGGL(KERNEL<0>, dim3(grid), blk, sm, st, ARGS);             \
  } while (0)

void launch_march(int precision, const MarchArgs& a, int grid, hipStream_t st) { DIST_DISPATCH(k_march, a); }
void launch_march_ring(int precision, const MarchArgs& a, int grid, hipStream_t st) { DIST_DISPATCH(k_march_ring, a); }
void launch_color(int precision, const ColorArgs& a, int grid, hipStream_t st) {
  const size_t sm = mlp_smem_bytes(precision, a.net);
  if (precision == 1) hipLaunchKernelGGL(k_color<1>, dim3(grid), dim3(kFwdWaves<1> * 64), sm, st, a);
  else if (precision == 0) hipLaunchKernelGGL(k_color<0>, dim3(grid), dim3(kFwdWaves<0> * 64), sm, st, a);
}
void launch_color_adjoint(int precision, const AdjArgs& a, int grid, hipStream_t st) {
  const size_t sm = mlp_smem_bytes(precision, a.net);
  if (precision == 2) hipLaunchKernelGGL(k_color_adjoint<2>, dim3(grid), dim3(kBwdWaves * 64), sm, st, a);
  else if (precision == 0) hipLaunchKernelGGL(k_color_adjoint<0>, dim3(grid), dim3(kBwdWaves * 64), sm, st, a);
}
void launch_eval(int precision, const EvalArgs& a, int grid, hipStream_t st) { DIST_DISPATCH(k_eval, a); }
void launch_adjoint(int precision, const AdjArgs& a, int grid, hipStream_t st) { DIST_DISPATCH_BWD(k_adjoint, a); }
static_assert(kAdjWaves * 64 == 512, "the recompute-and-VJP dispatch assumes 8 waves");
int mlp_row_groups(int waves, int width) { return (waves == 8 && width <= 128) ? 2 : 1; }
int adjoint_waves() { return kAdjWaves; }
int vjp_saved_waves(int precision) { return precision == 1 ? kVjpWaves<1> : kVjpWaves<0>; }
void launch_vjp_saved(int precision, const AdjArgs& a, int grid, hipStream_t st) {
  const size_t sm = mlp_smem_bytes(precision, a.net);
  if (precision == 1) hipLaunchKernelGGL(k_vjp_saved<1>, dim3(grid), dim3(kVjpWaves<1> * 64), sm, st, a);
  else if (precision == 2) hipLaunchKernelGGL(k_vjp_saved<2>, dim3(grid), dim3(kVjpWaves<2> * 64), sm, st, a);
  else if (precision == 0) hipLaunchKernelGGL(k_vjp_saved<0>, dim3(grid), dim3(kVjpWaves<0> * 64), sm, st, a);
}

// ---------------------------------------------------------------------------
// Weight packing into MFMA A-operand fragments.
//   bf16: fragment (rt, ks) = 64 lanes x 8 values, lane l holds row rt*32 + l%32,
//         columns ks*16 + (l/32)*8 + 0..7
//   f32 : fragment (rt, ks) = 64 lanes x 4 values, lane l holds row rt*32 + l%32,
//         columns ks*8 + (l/32)*4 + 0..3
// Rows are output features (or input features when transposed), columns the
// contracted dimension; entries outside the matrix are zero.
// ---------------------------------------------------------------------------
__global__ void k_pack(int precision, int transpose, const float* __restrict__ W, int out, int in_stride,
                       int ncols, int rows_pad, int cols_pad, void* dst) {
  const long long total = (long long)rows_pad * cols_pad;
  const int kfrag = precision ? 16 : 8;
  const int per = precision ? 8 : 4;
  const int ksteps = cols_pad / kfrag;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const int e = (int)(i % per);
    const long long fl = i / per;
    const int lane = (int)(fl % 64);
    const long long frag = fl / 64;
    const int ks = (int)(frag % ksteps);
    const int rt = (int)(frag / ksteps);
    const int row = rt * 32 + (lane & 31);
    const int col = ks * kfrag + (lane >> 5) * per + e;
    // matrix A[row][col]: W[row][col] or, transposed, W[col][row]
    const int n = transpose ? col : row;   // output feature of W
    const int k = transpose ? row : col;   // input feature of W (hidden part)
    float v = 0.f;
    if (n < out && k < ncols) v = W[(size_t)n * in_stride + k];
    if (precision == 2) v = v - (float)(bf16)v;          // low part of the split
    if (precision) ((bf16*)dst)[i] = (bf16)v;
    else ((float*)dst)[i] = v;
  }
}

void launch_pack_w(int precision, bool transpose, const float* W, int out, int in_stride, int ncols,
                   int npad, int kpad, void* dst, hipStream_t st) {
  // not transposed: rows = npad (outputs), cols = kpad (inputs); transposed: rows = kpad, cols = npad
  const int rows_pad = transpose ? kpad : npad;
  const int cols_pad = transpose ? npad : kpad;
  const long long total = (long long)rows_pad * cols_pad;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, st, precision, transpose ? 1 : 0, W, out, in_stride, ncols,
                     rows_pad, cols_pad, dst);
}

// Bias fragments (see acc_mfma_start): per 32-row tile, 64 lanes; lane l of
// tile t holds row t*32 + l%32 in its first column(s) if l < 32, zeros else.
__global__ void k_pack_bias(int precision, const float* __restrict__ bias, int n_tiles, void* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tiles * 64) return;
  const int tile = i >> 6, lane = i & 63;
  const float b = lane < 32 ? bias[tile * 32 + lane] : 0.f;
  if (precision == 0) {
    ((float*)dst)[i] = b;
  } else {
    const bf16 hi = (bf16)b;
    const float r1 = b - (float)hi;
    const bf16 mid = (bf16)r1;
    const bf16 lo = (bf16)(r1 - (float)mid);
    const bf16 z0 = (bf16)0.f;
    ((bf16x8*)dst)[i] = bf16x8{hi, mid, lo, z0, z0, z0, z0, z0};
  }
}

void launch_pack_bias(int precision, const float* bias, int wpad, void* dst, hipStream_t st) {
  const int n_tiles = wpad / 32;
  hipLaunchKernelGGL(k_pack_bias, dim3((n_tiles * 64 + 255) / 256), dim3(256), 0, st, precision, bias, n_tiles, dst);
}

// dst[l][n] = b[n] + sum_j Wz[n][j] z[l][j]  (rows n >= nout are zero)
__global__ void k_fold_bias(const float* __restrict__ b, const float* __restrict__ Wz, const float* __restrict__ z,
                            int n_lat, int L, int nout, int npad, float* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_lat * npad) return;
  const int l = i / npad, n = i - l * npad;
  float acc = 0.f;
  if (n < nout) {
    acc = b[n];
    const float* w = Wz + (size_t)n * L;
    const float* zz = z + (size_t)l * L;
    int j = 0;
    // 32 weights requested before the 32 products are summed in order
    for (; j + 32 <= L; j += 32) {
      float wv[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) wv[u] = w[j + u];
#pragma unroll
      for (int u = 0; u < 32; ++u) acc = fmaf(wv[u], zz[j + u], acc);
    }
    for (; j < L; ++j) acc = fmaf(w[j], zz[j], acc);
  }
  dst[i] = acc;
}

void launch_fold_bias(const float* b, const float* Wz, const float* z, int n_lat, int L, int nout, int npad,
                      float* dst, hipStream_t st) {
  const int total = n_lat * npad;
  hipLaunchKernelGGL(k_fold_bias, dim3((total + 255) / 256), dim3(256), 0, st, b, Wz, z, n_lat, L, nout, npad, dst);
}

}  // namespace dist
