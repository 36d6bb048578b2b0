// Ray bookkeeping kernels: generation and unit-sphere initialisation, the
// coarse-to-fine split, finalisation of the rendered
// maps, normals, and the gradient-sample list of the backward pass.  All of
// them are memory-bound (a few tens of bytes per ray) and use wave64 ballots
// with one atomic per workgroup for list appends.
#include "dist_internal.h"
#include "ray_kernels.h"

namespace dist {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Append `value` to list for every thread with flag set; one atomic per
// block of NT threads.  Must be called by all threads of the block.  Returns the
// list position of a flagged thread's entry (-1 for the others); the entry at
// position i is stored at list[dir * i], so dir = -1 fills backwards from the
// element `list` points at.
template <int NT = 256>
__device__ __forceinline__ int block_append(bool flag, int value, int* list, int* counter, int dir = 1) {
  __shared__ int wcnt[NT / 64];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int within = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) wcnt[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += wcnt[i];
    base = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  int off = base;
  for (int i = 0; i < w; ++i) off += wcnt[i];
  if (flag) list[dir * (off + within)] = value;
  __syncthreads();
  return flag ? off + within : -1;
}

// Level-`lvl` ray through the centre of block (U, V): unit world direction and
// the normalised image coordinates (xt, yt) = K^-1 (x, y) of that centre.
__device__ __forceinline__ void level_ray(const ImgDesc& im, int lvl, int U, int V, float3& d, float& xt, float& yt) {
  const float sc = (float)(1 << lvl);
  const float u = sc * (float)U + 0.5f * sc;
  const float v = sc * (float)V + 0.5f * sc;
  xt = (u - im.cx) / im.fx;
  yt = (v - im.cy) / im.fy;
  const float nrm = sqrtf(xt * xt + yt * yt + 1.f);
  const float a = xt / nrm, b = yt / nrm, c = 1.f / nrm;
  d.x = im.R[0] * a + im.R[1] * b + im.R[2] * c;
  d.y = im.R[3] * a + im.R[4] * b + im.R[5] * c;
  d.z = im.R[6] * a + im.R[7] * b + im.R[8] * c;
}

// Unit-sphere interval of the ray c + t d (Sec. 3.2 initialisation).
__device__ __forceinline__ bool sphere_interval(const ImgDesc& im, float3 d, float& t_lo, float& t_hi) {
  const float b = im.c[0] * d.x + im.c[1] * d.y + im.c[2] * d.z;
  const float cc = im.c[0] * im.c[0] + im.c[1] * im.c[1] + im.c[2] * im.c[2];
  const float disc = b * b - (cc - 1.f);
  const float sq = sqrtf(fmaxf(disc, 0.f));
  t_lo = fmaxf(-b - sq, im.near_);
  t_hi = fminf(-b + sq, im.far_);
  // the camera is outside the sphere, so both roots share a sign: the ray
  // meets the sphere only if they lie ahead of it (b < 0)
  return disc > 0.f && b < 0.f;
}

// Distance from the origin to the ray c + t v, t >= 0 (b = c . v): the foot of
// the perpendicular if it lies ahead, else the camera centre (App. A.3).
__device__ __forceinline__ float ray_origin_distance(float cc, float b) {
  return b < 0.f ? sqrtf(fmaxf(cc - b * b, 0.f)) : sqrtf(cc);
}

__device__ __forceinline__ void init_ray(const RayPool& pl, const ImgDesc& im, int img, int r, float3 d, float t,
                                         float t_lo, float t_hi, bool inside, int step) {
  pl.d[r] = make_float4(d.x, d.y, d.z, t);
  pl.b[r] = make_float2(t_lo, t_hi);
  pl.img[r] = img;
  pl.st[r] = inside ? ST_ACTIVE : ST_MISS;
  pl.n[r] = (uint8_t)step;
  pl.flast[r] = 0.f;
  for (int k = 0; k < im.K; ++k) {
    pl.rec_f[(size_t)k * pl.cap + r] = INFINITY;
    pl.rec_t[(size_t)k * pl.cap + r] = 0.f;
    pl.rec_n[(size_t)k * pl.cap + r] = 0;
  }
}

// ---------------------------------------------------------------------------
// Coarsest level: one ray per 2^L x 2^L block, starting at the sphere entry.
// grid: (blocks over rays of the largest image, n_images in `imgs_list`)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_level(RayPool pl, ImgDesc* imgs, const int* imgs_list,
                                                    int* list, int* counter) {
  const int img = imgs_list[blockIdx.y];
  const ImgDesc& im = imgs[img];
  const int lvl = im.levels;
  const int Wl = im.W >> lvl, Hl = im.H >> lvl;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  int r = 0;
  if (i < Wl * Hl) {
    const int V = i / Wl, U = i - V * Wl;
    float3 d;
    float xt, yt, t_lo, t_hi;
    level_ray(im, lvl, U, V, d, xt, yt);
    const bool inside = sphere_interval(im, d, t_lo, t_hi);
    r = im.slot_base + im.lvl_off[lvl] + i;
    init_ray(pl, im, img, r, d, t_lo, t_lo, t_hi, inside, 0);
    act = inside;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) imgs[img].cur_level = lvl;
  block_append(act, r, list, counter);
}

// ---------------------------------------------------------------------------
// Coarse-to-fine split (Sec. 3.2, Fig. 3a): every ray of level lvl+1 becomes
// four rays of level lvl.  A child starts from the parent's t clamped into its
// own unit-sphere interval (from its own entry if the parent missed) and is
// re-activated whatever the parent's state; its records start empty.
// With counter_tail the list is filled from both ends: children of rays still
// marching at the split (the ones that need the most further steps) from the
// front, the others backwards from list[tail_end - 1], so a consumer that
// takes the rays in order starts the long ones first.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_split(RayPool pl, ImgDesc* imgs, const int* imgs_list, int child_lvl,
                                               int child_step, int* list, int* counter, int* counter_tail,
                                               int tail_end) {
  const int img = imgs_list[blockIdx.y];
  const ImgDesc& im = imgs[img];
  const int Wl = im.W >> child_lvl, Hl = im.H >> child_lvl;
  const int Wp = im.W >> (child_lvl + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false, marching = false;
  int r = 0;
  if (i < Wl * Hl) {
    const int V = i / Wl, U = i - V * Wl;
    float3 d;
    float xt, yt, t_lo, t_hi;
    level_ray(im, child_lvl, U, V, d, xt, yt);
    const bool inside = sphere_interval(im, d, t_lo, t_hi);
    const int pr = im.slot_base + im.lvl_off[child_lvl + 1] + (V >> 1) * Wp + (U >> 1);
    const uint8_t pst = pl.st[pr];
    const float tp = pst == ST_MISS ? t_lo : pl.d[pr].w;
    const float t = fminf(fmaxf(tp, t_lo), t_hi);
    r = im.slot_base + im.lvl_off[child_lvl] + i;
    init_ray(pl, im, img, r, d, t, t_lo, t_hi, inside, child_step);
    act = inside;
    marching = pst == ST_ACTIVE;
  }
  // 1024-thread blocks: a quarter of the atomics on the list counters
  if (counter_tail) {
    block_append<1024>(act && marching, r, list, counter);
    block_append<1024>(act && !marching, r, list + tail_end - 1, counter_tail, -1);
  } else {
    block_append<1024>(act, r, list, counter);
  }
}

__global__ void k_set_level(ImgDesc* imgs, const int* imgs_list, int n, int lvl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) imgs[imgs_list[i]].cur_level = lvl;
}

// ---------------------------------------------------------------------------
// Finalise level-0 rays into the output maps (Sec. 3.3, App. A.3).
// grid: (1024-pixel blocks over H*W, n_images); one list atomic per block
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_finalize(RayPool pl, const ImgDesc* imgs, const int* imgs_list,
                                                  FinalizeOut o) {
  const int img = imgs_list ? imgs_list[blockIdx.y] : blockIdx.y;
  const ImgDesc& im = imgs[img];
  const int hw = im.H * im.W;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  int r = 0;
  if (pix < hw) {
    r = im.slot_base + im.lvl_off[0] + pix;
    const uint8_t st = pl.st[r];
    const size_t q = (size_t)im.out_base + pix;
    const int V = pix / im.W, U = pix - V * im.W;
    float3 dd;
    float xt, yt;
    level_ray(im, 0, U, V, dd, xt, yt);
    const float4 d = pl.d[r];
    hit = st == ST_HIT;
    float depth = INFINITY, dist = INFINITY, sil;
    if (hit) {
      dist = d.w + pl.flast[r];
      depth = dist / sqrtf(xt * xt + yt * yt + 1.f);
    }
    if (st == ST_MISS) {
      const float b = im.c[0] * d.x + im.c[1] * d.y + im.c[2] * d.z;
      const float cc = im.c[0] * im.c[0] + im.c[1] * im.c[1] + im.c[2] * im.c[2];
      sil = ray_origin_distance(cc, b) - 1.f;
    } else if (st == ST_ERROR) {
      sil = INFINITY;                      // a non-finite query: background
    } else {
      sil = fabsf(pl.rec_f[r]) - im.eps;
    }
    if (o.depth) o.depth[q] = depth;
    if (o.dist) o.dist[q] = dist;
    if (o.sil) o.sil[q] = sil;
    if (o.status) o.status[q] = st;
    if (o.nsteps) o.nsteps[q] = st == ST_MISS ? 0 : pl.n[r];
    if (o.normal && !hit) { o.normal[3 * q] = 0.f; o.normal[3 * q + 1] = 0.f; o.normal[3 * q + 2] = 0.f; }
    if (o.nraw) o.nraw[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int h = block_append<1024>(hit && o.want_hits, r, o.hits, o.hit_count);
  if (o.hit_pix && pix < hw) o.hit_pix[(size_t)im.out_base + pix] = h;
}

// Normals from the six central-difference queries of each hit (Sec. 3.3).
__global__ void k_normals(const RayPool pl, const ImgDesc* imgs, const int* hits, const int* hit_count,
                          const float* fv, float delta, float* normal, float4* nraw) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= *hit_count) return;
  const int r = hits[h];
  const ImgDesc& im = imgs[pl.img[r]];
  const int pix = r - im.slot_base - im.lvl_off[0];
  const size_t q = (size_t)im.out_base + pix;
  const float* f = fv + 6ll * h;
  const float inv = 1.f / (2.f * delta);
  const float nx = (f[0] - f[1]) * inv, ny = (f[2] - f[3]) * inv, nz = (f[4] - f[5]) * inv;
  const float len = sqrtf(nx * nx + ny * ny + nz * nz);
  if (nraw) nraw[q] = make_float4(nx, ny, nz, len);
  if (normal) {
    const float s = len > 0.f ? 1.f / len : 0.f;
    normal[3 * q] = nx * s;
    normal[3 * q + 1] = ny * s;
    normal[3 * q + 2] = nz * s;
  }
}

// ---------------------------------------------------------------------------
// Backward: gradient samples (Sec. 3.4 Eq. 2 first term; App. B.2)
// ---------------------------------------------------------------------------
struct PixSamples {
  int nd, base, nn;      // depth records used, samples at records, normal samples
};

__device__ __forceinline__ PixSamples pixel_samples(const RayPool& pl, const ImgDesc& im, int r, size_t q,
                                                    const SeedIn& in) {
  PixSamples ps{0, 0, 0};
  const uint8_t st = pl.st[r];
  if (st == ST_MISS || st == ST_ERROR) return ps;     // no samples on a ray that met a non-finite query
  const float gd = in.g_depth ? in.g_depth[q] : 0.f;
  const float gs = in.g_sil ? in.g_sil[q] : 0.f;
  if (in.hit_mode) {
    ps.base = (st == ST_HIT && gd != 0.f) ? 1 : 0;
    return ps;
  }
  if (in.imp_gv) {
    // silhouette sample at the minimum-|f| query, depth sample at the Eq. 1 point
    ps.base = ((gs != 0.f && pl.rec_f[r] != INFINITY) ? 1 : 0) + ((st == ST_HIT && gd != 0.f && in.imp_gv[q] != 0.f) ? 1 : 0);
  } else if (st == ST_HIT && gd != 0.f) {
    for (int k = 0; k < im.K; ++k) ps.nd += (pl.rec_f[(size_t)k * pl.cap + r] != INFINITY) ? 1 : 0;
  }
  if (!in.imp_gv) {
    const int ns = (gs != 0.f && pl.rec_f[r] != INFINITY) ? 1 : 0;
    ps.base = ps.nd > ns ? ps.nd : ns;
  }
  if (st == ST_HIT && in.g_normal && in.nraw) {
    const float* g = in.g_normal + 3 * q;
    if ((g[0] != 0.f || g[1] != 0.f || g[2] != 0.f) && in.nraw[q].w > 0.f) ps.nn = 6;
  }
  return ps;
}

// Per block of 256 pixels: the number of gradient samples.  With bsum2 (the
// split layout) the record samples and the normal-stencil samples are counted
// for two separate lists; otherwise a pixel's stencil samples follow its
// record samples in one list.
__global__ __launch_bounds__(256) void k_samples_count(RayPool pl, const ImgDesc* imgs, const int* img_order,
                                                       SeedIn in, int* bsum, int* bsum2) {
  __shared__ int red[256], red2[256];
  const int img = img_order[blockIdx.y];
  const ImgDesc& im = imgs[img];
  const int hw = im.H * im.W;
  const int pix = blockIdx.x * 256 + threadIdx.x;
  int c = 0, c2 = 0;
  if (pix < hw) {
    const PixSamples ps = pixel_samples(pl, im, im.slot_base + im.lvl_off[0] + pix, (size_t)im.out_base + pix, in);
    c = bsum2 ? ps.base : ps.base + ps.nn;
    c2 = ps.nn;
  }
  red[threadIdx.x] = c;
  red2[threadIdx.x] = c2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      red2[threadIdx.x] += red2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bsum[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
    if (bsum2) bsum2[blockIdx.y * gridDim.x + blockIdx.x] = red2[0];
  }
}

// One workgroup: exclusive scan of the block sums in image order, restarting
// the padding at every latent segment so that each segment starts at a
// multiple of the adjoint tile.  seg_* are indexed by latent id.  The list
// starts at *pos0 (0 if null); n_out[0] receives its end, n_out[1] its length.
__global__ __launch_bounds__(1024) void k_samples_scan(const int* bsum, int n_img, int bpi, const int* img_order,
                                                       const int* img_latent, int lat_fixed, int tile, int n_lat,
                                                       int* boff, int* seg_base, int* seg_total, int* seg_padded,
                                                       const int* pos0, int* n_out) {
  __shared__ int buf[1024];
  __shared__ int carry_s;
  const int tid = threadIdx.x;
  const int start = pos0 ? *pos0 : 0;
  for (int l = tid; l < n_lat; l += 1024) { seg_base[l] = start; seg_total[l] = 0; seg_padded[l] = 0; }
  __syncthreads();
  int pos = start;          // running padded offset (uniform)
  int i0 = 0;
  while (i0 < n_img) {
    const int lat = img_latent ? img_latent[img_order[i0]] : lat_fixed;
    int i1 = i0;
    while (i1 < n_img && (img_latent ? img_latent[img_order[i1]] : lat_fixed) == lat) ++i1;
    // scan blocks of images [i0, i1)
    const int nb = (i1 - i0) * bpi;
    const int b0 = i0 * bpi;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
      const int v = (c0 + tid < nb) ? bsum[b0 + c0 + tid] : 0;
      buf[tid] = v;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {
        const int x = tid >= off ? buf[tid - off] : 0;
        __syncthreads();
        buf[tid] += x;
        __syncthreads();
      }
      const int carry = carry_s;
      if (c0 + tid < nb) boff[b0 + c0 + tid] = pos + carry + buf[tid] - v;
      __syncthreads();
      if (tid == 1023) carry_s = carry + buf[1023];
      __syncthreads();
    }
    const int total = carry_s;
    const int padded = (total + tile - 1) / tile * tile;
    if (tid == 0) { seg_base[lat] = pos; seg_total[lat] = total; seg_padded[lat] = padded; }
    pos += padded;
    i0 = i1;
    __syncthreads();
  }
  if (tid == 0) {
    n_out[0] = pos;
    n_out[1] = pos - start;
  }
}

// Block-wide exclusive prefix of c over the 256 threads (all threads call).
__device__ __forceinline__ int block_excl_scan(int c, int* buf) {
  buf[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int x = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += x;
    __syncthreads();
  }
  return buf[threadIdx.x] - c;
}

// Writes each pixel's samples at the offsets of the scans.  With boff2 (split
// layout) the stencil samples go to the second list, each with its stencil
// index 6 h + j (h = the pixel's hit index in the forward's hit list), so that
// their adjoint can use the masks the forward kept.
__global__ __launch_bounds__(256) void k_samples_write(RayPool pl, const ImgDesc* imgs, const int* img_order,
                                                       SeedIn in, const int* boff, const int* boff2, float4* samples,
                                                       int* sample_lat, int* sample_idx, int4* sample_cam) {
  __shared__ int buf[256];
  const int img = img_order[blockIdx.y];
  const ImgDesc& im = imgs[img];
  const int hw = im.H * im.W;
  const int pix = blockIdx.x * 256 + threadIdx.x;
  PixSamples ps{0, 0, 0};
  int r = 0;
  size_t q = 0;
  if (pix < hw) {
    r = im.slot_base + im.lvl_off[0] + pix;
    q = (size_t)im.out_base + pix;
    ps = pixel_samples(pl, im, r, q, in);
  }
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  const int c = boff2 ? ps.base : ps.base + ps.nn;
  int o = boff[blk] + block_excl_scan(c, buf);
  int o2 = 0;
  if (boff2) {
    __syncthreads();
    o2 = boff2[blk] + block_excl_scan(ps.nn, buf);
  }
  if (ps.base + ps.nn == 0) return;
  const float4 d = pl.d[r];
  const float cx = im.c[0], cy = im.c[1], cz = im.c[2];
  const int V = pix / im.W, U = pix - V * im.W;
  float3 dd;
  float xt, yt;
  level_ray(im, 0, U, V, dd, xt, yt);
  const float gd = in.g_depth ? in.g_depth[q] : 0.f;
  const float gs = in.g_sil ? in.g_sil[q] : 0.f;
  const float dseed = im.alpha * gd / sqrtf(xt * xt + yt * yt + 1.f);
  const float dist_eq1 = d.w + pl.flast[r];
  if (in.hit_mode || in.imp_gv) {
    const float f0 = pl.rec_f[r];
    if (in.imp_gv && gs != 0.f && f0 != INFINITY) {
      const float t0 = pl.rec_t[r];
      samples[o] = make_float4(fmaf(t0, d.x, cx), fmaf(t0, d.y, cy), fmaf(t0, d.z, cz),
                               gs * (f0 > 0.f ? 1.f : (f0 < 0.f ? -1.f : 0.f)));
      sample_lat[o] = im.latent;
      if (sample_cam) sample_cam[o] = make_int4(img, pix, __float_as_int(t0), 0);
      ++o;
    }
    const bool dep = pl.st[r] == ST_HIT && gd != 0.f && (in.hit_mode || in.imp_gv[q] != 0.f);
    if (dep) {
      const float seed = in.hit_mode ? 1.f : -gd / sqrtf(xt * xt + yt * yt + 1.f) / in.imp_gv[q];
      samples[o] = make_float4(fmaf(dist_eq1, d.x, cx), fmaf(dist_eq1, d.y, cy), fmaf(dist_eq1, d.z, cz), seed);
      sample_lat[o] = im.latent;
      if (sample_cam) sample_cam[o] = make_int4(img, pix, __float_as_int(dist_eq1), 0);
      ++o;
    }
  }
  for (int k = 0; k < ((in.hit_mode || in.imp_gv) ? 0 : ps.base); ++k) {
    const float tk = pl.rec_t[(size_t)k * pl.cap + r];
    float seed = k < ps.nd ? dseed : 0.f;
    if (k == 0 && gs != 0.f) {
      const float f0 = pl.rec_f[r];
      seed += gs * (f0 > 0.f ? 1.f : (f0 < 0.f ? -1.f : 0.f));
    }
    samples[o] = make_float4(fmaf(tk, d.x, cx), fmaf(tk, d.y, cy), fmaf(tk, d.z, cz), seed);
    sample_lat[o] = im.latent;
    if (sample_cam) sample_cam[o] = make_int4(img, pix, __float_as_int(tk), 0);
    ++o;
  }
  if (ps.nn) {
    const float4 nr = in.nraw[q];
    const float inv = 1.f / nr.w;
    const float nx = nr.x * inv, ny = nr.y * inv, nz = nr.z * inv;
    const float* g = in.g_normal + 3 * q;
    const float gn = g[0] * nx + g[1] * ny + g[2] * nz;
    const float gv[3] = {(g[0] - gn * nx) * inv, (g[1] - gn * ny) * inv, (g[2] - gn * nz) * inv};
    const float dist = d.w + pl.flast[r];
    const float p[3] = {fmaf(dist, d.x, cx), fmaf(dist, d.y, cy), fmaf(dist, d.z, cz)};
    const float s2 = 1.f / (2.f * in.delta);
    const int h = boff2 ? in.hit_pix[q] : 0;
    for (int j = 0; j < 6; ++j) {
      const int ax = j >> 1;
      float qv[3] = {p[0], p[1], p[2]};
      qv[ax] = (j & 1) ? qv[ax] - in.delta : qv[ax] + in.delta;
      const float seed = (j & 1) ? -gv[ax] * s2 : gv[ax] * s2;
      const int at = boff2 ? o2++ : o++;
      samples[at] = make_float4(qv[0], qv[1], qv[2], seed);
      sample_lat[at] = im.latent;
      if (boff2) sample_idx[at] = 6 * h + j;
    }
  }
}

// Padding samples (zero seed) at the end of each latent segment; their
// stencil index (split layout) is 0, a valid entry whose contribution the zero
// seed cancels.
__global__ void k_samples_pad(const int* seg_base, const int* seg_total, const int* seg_padded, float4* samples,
                              int* sample_lat, int* sample_idx, int4* sample_cam) {
  const int l = blockIdx.x;
  const int b = seg_base[l], t = seg_total[l], p = seg_padded[l];
  for (int i = t + threadIdx.x; i < p; i += blockDim.x) {
    samples[b + i] = make_float4(0.f, 0.f, 0.f, 0.f);
    sample_lat[b + i] = l;
    if (sample_idx) sample_idx[b + i] = 0;
    if (sample_cam) sample_cam[b + i] = make_int4(-1, 0, 0, 0);
  }
}

// Camera-extrinsic gradient of one view (blockIdx.x), fixed summation order:
// every depth/silhouette sample of the view's images adds s grad_p f(p) to
// dL/dc and s t grad_p f(p) u^T to dL/dR (p = c + t R u, t detached), with
// s grad_p f = s 0.5 p/|p| + the adjoint's per-wave partials; every pixel whose
// ray misses the unit sphere adds dL/dS dS/d(c, R) of S = sqrt(|c|^2 -
// (c.v)^2) - 1 (App. A.3).  Output g_cam[v] = (dL/dc, dL/dR row-major).
__global__ __launch_bounds__(256) void k_cam_reduce(RayPool pl, const ImgDesc* imgs, const int* img_view, int n_img,
                                                    const float4* samples, const int4* sample_cam,
                                                    const float* gp_part, const int* n_samples, const float* g_sil,
                                                    float* g_cam) {
  __shared__ float red[256];
  const int v = blockIdx.x;
  float acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.f;
  const int ns = *n_samples;
  for (int i = threadIdx.x; i < ns; i += 256) {
    const int4 sc = sample_cam[i];
    if (sc.x < 0 || img_view[sc.x] != v) continue;
    const ImgDesc& im = imgs[sc.x];
    const float4 smp = samples[i];
    const float rn = sqrtf(smp.x * smp.x + smp.y * smp.y + smp.z * smp.z);
    const float h = rn > 0.f ? 0.5f * smp.w / rn : 0.f;
    float g[3] = {h * smp.x, h * smp.y, h * smp.z};
    const float* pp = gp_part + (size_t)i * 3 * kGpSlots;
    for (int w = 0; w < kGpSlots; ++w) {
      g[0] += pp[3 * w];
      g[1] += pp[3 * w + 1];
      g[2] += pp[3 * w + 2];
    }
    const int V = sc.y / im.W, U = sc.y - V * im.W;
    float3 d;
    float xt, yt;
    level_ray(im, 0, U, V, d, xt, yt);
    const float nrm = sqrtf(xt * xt + yt * yt + 1.f);
    const float u[3] = {xt / nrm, yt / nrm, 1.f / nrm};
    const float t = __int_as_float(sc.z);
    for (int a = 0; a < 3; ++a) {
      acc[a] += g[a];
      for (int b = 0; b < 3; ++b) acc[3 + 3 * a + b] = fmaf(g[a] * t, u[b], acc[3 + 3 * a + b]);
    }
  }
  if (g_sil) {
    for (int img = 0; img < n_img; ++img) {
      if (img_view[img] != v) continue;
      const ImgDesc& im = imgs[img];
      const int hw = im.H * im.W;
      for (int pix = threadIdx.x; pix < hw; pix += 256) {
        const int r = im.slot_base + im.lvl_off[0] + pix;
        const float gs = g_sil[(size_t)im.out_base + pix];
        if (pl.st[r] != ST_MISS || gs == 0.f) continue;
        const int V = pix / im.W, U = pix - V * im.W;
        float3 d;
        float xt, yt;
        level_ray(im, 0, U, V, d, xt, yt);
        const float nrm = sqrtf(xt * xt + yt * yt + 1.f);
        const float u[3] = {xt / nrm, yt / nrm, 1.f / nrm};
        const float c[3] = {im.c[0], im.c[1], im.c[2]};
        const float dv[3] = {d.x, d.y, d.z};
        const float b0 = c[0] * dv[0] + c[1] * dv[1] + c[2] * dv[2];
        // S = (distance from the origin to the ray) - 1: with the foot of the
        // perpendicular behind the camera it is |c| - 1 (b enters as 0)
        const float b = b0 < 0.f ? b0 : 0.f;
        const float q = ray_origin_distance(c[0] * c[0] + c[1] * c[1] + c[2] * c[2], b0);
        if (!(q > 0.f)) continue;
        const float w = gs / q;
        for (int a = 0; a < 3; ++a) {
          acc[a] = fmaf(w, c[a] - b * dv[a], acc[a]);
          const float da = -w * b * c[a];
          for (int bb = 0; bb < 3; ++bb) acc[3 + 3 * a + bb] = fmaf(da, u[bb], acc[3 + 3 * a + bb]);
        }
      }
    }
  }
  // fixed-order tree reduction of each of the 12 sums
  for (int k = 0; k < 12; ++k) {
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) g_cam[12 * v + k] = red[0];
    __syncthreads();
  }
}

// g_z[l] = W0_z^T S0 + Ws_z^T Ss with S = sum over the latent's tiles.  The
// sum runs in two fixed-order passes: k_gz_fold adds each run of 64 tiles into
// the run's first tile, k_gz_reduce adds the run heads and applies W_z^T.
// Bitwise reproducible.
// Both keep several tiles' loads in flight per thread (the chains are bound by
// memory latency, not bandwidth) and add them in tile order.
constexpr int kFold = 64;

__global__ __launch_bounds__(512) void k_gz_fold(float* partial, int kmax, int tile, const int* seg_base,
                                                 const int* seg_padded, int lat0) {
  const int l = lat0 + blockIdx.y;
  const int t0 = seg_base[l] / tile, nt = seg_padded[l] / tile;
  const int c0 = blockIdx.x * kFold;
  if (c0 >= nt) return;
  const int c1 = min(c0 + kFold, nt);
  const int width = 4 * kmax;
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    const float* p = partial + (size_t)(t0 + c0) * width + i;
    float a = 0.f;
    int t = 0;
    for (; t + 8 <= c1 - c0; t += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(t + u) * width];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; t < c1 - c0; ++t) a += p[(size_t)t * width];
    partial[(size_t)(t0 + c0) * width + i] = a;
  }
}

// One workgroup per latent.  The run heads of a column are summed in two
// halves (each in head order, added half 0 + half 1), and each output of the
// latent code in four quarters of the contracted rows [W0_z; Ws_z] (each in
// row order, added in quarter order), so every chain is short and the order
// is fixed.
__global__ __launch_bounds__(1024) void k_gz_reduce(const float* partial, int kmax, int tile, const int* seg_base,
                                                    const int* seg_padded, int w0, int mg0, const float* W0z,
                                                    int ws, int mgs, const float* Wsz, int L, float* gz, int lat0,
                                                    int accumulate) {
  __shared__ float S0[512];
  __shared__ float Ss[512];
  __shared__ float ph[2][2][512];
  __shared__ float pq[4][256];
  const int l = lat0 + blockIdx.x;
  const int t0 = seg_base[l] / tile, nt = seg_padded[l] / tile;
  const int nheads = (nt + kFold - 1) / kFold;
  {
    const int half = threadIdx.x >> 9, n = threadIdx.x & 511;
    const int h1 = half ? nheads : nheads / 2;
    int h = half ? nheads / 2 : 0;
    float a = 0.f, b = 0.f;
    for (; h + 4 <= h1; h += 4) {
      float va[4][2], vb[4][2];            // four run heads (up to two row groups each) in flight
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* pt = partial + (size_t)(t0 + (h + u) * kFold) * 4 * kmax;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          va[u][g] = (g < mg0 && n < w0) ? pt[g * kmax + n] : 0.f;
          vb[u][g] = (Wsz && g < mgs && n < ws) ? pt[(2 + g) * kmax + n] : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        for (int g = 0; g < mg0; ++g) a += va[u][g];
        if (Wsz)
          for (int g = 0; g < mgs; ++g) b += vb[u][g];
      }
    }
    for (; h < h1; ++h) {
      const float* pt = partial + (size_t)(t0 + h * kFold) * 4 * kmax;
      for (int g = 0; g < mg0; ++g) a += (n < w0) ? pt[g * kmax + n] : 0.f;
      if (Wsz)
        for (int g = 0; g < mgs; ++g) b += (n < ws) ? pt[(2 + g) * kmax + n] : 0.f;
    }
    ph[0][half][n] = a;
    ph[1][half][n] = b;
  }
  __syncthreads();
  if (threadIdx.x < 512) {
    S0[threadIdx.x] = ph[0][0][threadIdx.x] + ph[0][1][threadIdx.x];
    Ss[threadIdx.x] = ph[1][0][threadIdx.x] + ph[1][1][threadIdx.x];
  }
  __syncthreads();
  const int q = threadIdx.x >> 8, jl = threadIdx.x & 255;
  const int rows = w0 + (Wsz ? ws : 0);
  const int r0 = q * rows / 4, r1 = (q + 1) * rows / 4;
  for (int j0 = 0; j0 < L; j0 += 256) {
    const int j = j0 + jl;
    float acc = 0.f;
    if (j < L) {
      int r = r0;
      for (; r + 8 <= r1; r += 8) {
        float w[8], x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = r + u;
          w[u] = rr < w0 ? W0z[(size_t)rr * L + j] : Wsz[(size_t)(rr - w0) * L + j];
          x[u] = rr < w0 ? S0[rr] : Ss[rr - w0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fmaf(w[u], x[u], acc);
      }
      for (; r < r1; ++r)
        acc = fmaf(r < w0 ? W0z[(size_t)r * L + j] : Wsz[(size_t)(r - w0) * L + j], r < w0 ? S0[r] : Ss[r - w0], acc);
    }
    pq[q][jl] = acc;
    __syncthreads();
    if (q == 0 && j < L) {
      const float v = ((pq[0][jl] + pq[1][jl]) + pq[2][jl]) + pq[3][jl];
      gz[(size_t)l * L + j] = accumulate ? gz[(size_t)l * L + j] + v : v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Serving: the next pooled active list is built from (a) the rays still active
// in the previous list and then (b) the children of images that split this
// tick and the coarsest rays of newly (re)started images, counting per image
// the rays it has in the new list.  (a) and (b) are separate launches: a ray
// slot released by a finished request can be handed to a request that starts
// this tick while the previous list still names it, and the stale entry must
// be read (and dropped, its ray having stopped) before the slot is
// re-initialised.
// ---------------------------------------------------------------------------
__global__ void k_apply_levels(ImgDesc* imgs, const AdvEntry* table, const int* hdr) {
  const int n = hdr[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    imgs[table[i].img].cur_level = table[i].lvl;
}

// per-image count of the wave's flagged entries: one atomic per distinct image
__device__ __forceinline__ void count_per_image(bool flag, int img, int* img_active) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(flag);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int li = __shfl(img, leader);
    const unsigned long long same = __ballot(flag && img == li);
    if (lane == leader) atomicAdd(&img_active[li], __popcll(same));
    todo &= ~same;
  }
}

__global__ __launch_bounds__(256) void k_advance_old(RayPool pl, const ImgDesc* imgs, const int* in_list,
                                                     const int* in_count, int* out_list, int* out_count,
                                                     int* img_active) {
  const int n_old = *in_count;
  for (int base = blockIdx.x * 256; base < n_old; base += gridDim.x * 256) {
    const int i = base + threadIdx.x;
    bool keep = false;
    int r = 0, img = -1;
    if (i < n_old) {
      r = in_list[i];
      if (pl.st[r] == ST_ACTIVE) {
        img = pl.img[r];
        const ImgDesc& im = imgs[img];
        const int off = r - im.slot_base;
        const int hw = im.H * im.W;
        const int lvl = off < hw ? 0 : (off < hw + (hw >> 2) ? 1 : 2);
        keep = lvl == im.cur_level;
      }
    }
    count_per_image(keep, img, img_active);
    block_append(keep, r, out_list, out_count);
  }
}

__global__ __launch_bounds__(256) void k_advance_new(RayPool pl, const ImgDesc* imgs, int* out_list, int* out_count,
                                                     const AdvEntry* table, const int* hdr, int* img_active) {
  const int n_tab = hdr[0], n_new = hdr[1];
  for (int base = blockIdx.x * 256; base < n_new; base += gridDim.x * 256) {
    const int j = base + threadIdx.x;
    bool keep = false;
    int r = 0, img = -1;
    if (j < n_new) {
      int lo = 0, hi = n_tab - 1;          // last entry with begin <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].begin <= j) lo = mid; else hi = mid - 1;
      }
      const AdvEntry e = table[lo];
      img = e.img;
      const ImgDesc& im = imgs[img];
      const int c = j - e.begin;
      const int lvl = e.lvl;
      const int Wl = im.W >> lvl;
      const int V = c / Wl, U = c - V * Wl;
      float3 d;
      float xt, yt, t_lo, t_hi;
      level_ray(im, lvl, U, V, d, xt, yt);
      const bool inside = sphere_interval(im, d, t_lo, t_hi);
      float t = t_lo;
      if (e.split) {
        const int Wp = im.W >> (lvl + 1);
        const int pr = im.slot_base + im.lvl_off[lvl + 1] + (V >> 1) * Wp + (U >> 1);
        const float tp = pl.st[pr] == ST_MISS ? t_lo : pl.d[pr].w;
        t = fminf(fmaxf(tp, t_lo), t_hi);
      }
      r = im.slot_base + im.lvl_off[lvl] + c;
      init_ray(pl, im, img, r, d, t, t_lo, t_hi, inside, e.step);
      keep = inside;
    }
    count_per_image(keep, img, img_active);
    block_append(keep, r, out_list, out_count);
  }
}

// Image-space loss of inverse optimisation and its gradient w.r.t. the
// rendered maps, one workgroup per image (fixed summation order, no atomics):
//   L_i = 1/HW [ w_d sum_{fg_r & fg_t} |z_c - z_c*|                 (Sec. 4.2.1 L1 depth)
//              + w_s sum_pix S* max(0, S) + (1 - S*) max(0, -S)     (App. A.3 hinge)
//              + w_n sum_{fg_r & fg_t} (-n . n*) ]                  (App. B.3 normal term)
// fg_r: S < 0 (the rendered binary silhouette), fg_t: S* > 0.5.  sign(0) = 0
// and max'(0) = 0; a hinge term whose weight S* or 1 - S* is zero adds
// nothing.  Gradient outputs may be null (not written); normals are read
// only when w_n != 0.
__global__ __launch_bounds__(1024) void k_render_loss(const float* depth, const float* normal, const float* sil,
                                                      const float* depth_t, const float* normal_t,
                                                      const float* sil_t, int hw, float w_d, float w_s, float w_n,
                                                      float* loss, float* g_depth, float* g_normal, float* g_sil) {
  __shared__ float red[1024];
  const size_t base = (size_t)blockIdx.x * hw;
  const float inv = 1.f / (float)hw;
  const float cd = w_d * inv, cs = w_s * inv, cn = w_n * inv;
  const bool nrm = w_n != 0.f;
  float acc = 0.f;
  for (int p = threadIdx.x; p < hw; p += 1024) {
    const size_t i = base + p;
    const float S = sil[i], St = sil_t[i];
    const bool fg = S < 0.f && St > 0.5f;
    const float dd = fg ? depth[i] - depth_t[i] : 0.f;
    float l = cd * fabsf(dd);
    l += cs * ((St > 0.f ? St * fmaxf(S, 0.f) : 0.f) + (St < 1.f ? (1.f - St) * fmaxf(-S, 0.f) : 0.f));
    float nt[3] = {0.f, 0.f, 0.f};
    if (nrm && fg) {
      for (int k = 0; k < 3; ++k) nt[k] = normal_t[3 * i + k];
      l -= cn * (normal[3 * i] * nt[0] + normal[3 * i + 1] * nt[1] + normal[3 * i + 2] * nt[2]);
    }
    if (g_depth) g_depth[i] = cd * (dd > 0.f ? 1.f : (dd < 0.f ? -1.f : 0.f));
    if (g_sil) g_sil[i] = cs * (St * (S > 0.f ? 1.f : 0.f) - (1.f - St) * (S < 0.f ? 1.f : 0.f));
    if (g_normal)
      for (int k = 0; k < 3; ++k) g_normal[3 * i + k] = -cn * nt[k];
    acc += l;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[blockIdx.x] = red[0];
}

// out[0] = sum of a[0..n) in index order (one thread).
__global__ void k_sum_ordered(const float* a, int n, float* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += a[i];
    out[0] = s;
  }
}

// Adam (paper App. B.4: Adam, learning rate 1e-2) on one latent code.
__global__ void k_adam(float* z, float* m, float* v, const float* g, int L, float lr, float b1, float b2, float eps,
                       int t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  const float mh = mj / (1.f - powf(b1, (float)t));
  const float vh = vj / (1.f - powf(b2, (float)t));
  z[j] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_fill_i32(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Exact gradient through the unrolled march (Eq. 2 with both terms), in
// reverse over the marching steps.  lam[r] is the adjoint of ray r's current
// t: dL/dt after the step being processed.  A ray's query at step n gets the
// seed
//   a = alpha lam[r]            if the step moved t (t += alpha f)
//     + dL/dd / |(xt, yt, 1)|   at a level-0 hit's last step (d = t + f)
//     + dL/dS sign f            at a level-0 ray's minimum-|f| step,
// the decoder's VJP at that point adds a df/dz to dL/dz, and lam[r] gains
// a grad_p f . v (the same query's dependence on t through p = c + t v).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ul_seed(const RayPool& pl, const ImgDesc& im, int r, int pix, const UlIn& in) {
  const uint8_t st = pl.st[r];
  if (st == ST_MISS || st == ST_ERROR) return 0.f;
  const int last = (int)pl.n[r] - 1;
  if (in.step > last) return 0.f;
  const bool term = in.step == last;
  const bool moved = !(term && (st == ST_HIT || st == ST_UNCONVERGED));
  float a = moved ? im.alpha * in.lam[r] : 0.f;
  if (in.lvl == 0) {
    const size_t q = (size_t)im.out_base + pix;
    if (term && st == ST_HIT && in.g_depth) {
      const int V = pix / im.W, U = pix - V * im.W;
      float3 dd;
      float xt, yt;
      level_ray(im, 0, U, V, dd, xt, yt);
      a += in.g_depth[q] / sqrtf(xt * xt + yt * yt + 1.f);
    }
    if (in.g_sil && (int)pl.rec_n[r] == in.step && pl.rec_f[r] != INFINITY) {
      const float f0 = pl.rec_f[r];
      a += in.g_sil[q] * (f0 > 0.f ? 1.f : (f0 < 0.f ? -1.f : 0.f));
    }
  }
  return a;
}

// Per block of 256 rays of level in.lvl: the number of rays with a nonzero seed.
__global__ __launch_bounds__(256) void k_ul_count(RayPool pl, const ImgDesc* imgs, const int* img_order, UlIn in,
                                                  int* bsum) {
  __shared__ int red[256];
  const ImgDesc& im = imgs[img_order[blockIdx.y]];
  const int nr = (im.H >> in.lvl) * (im.W >> in.lvl);
  const int i = blockIdx.x * 256 + threadIdx.x;
  int c = 0;
  if (i < nr) c = ul_seed(pl, im, im.slot_base + im.lvl_off[in.lvl] + i, i, in) != 0.f ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Writes one sample per counted ray: its point of step in.step and its seed;
// sample_cam = (image, ray slot).
__global__ __launch_bounds__(256) void k_ul_write(RayPool pl, const ImgDesc* imgs, const int* img_order, UlIn in,
                                                  const int* boff, float4* samples, int* sample_lat,
                                                  int4* sample_cam) {
  __shared__ int buf[256];
  const int img = img_order[blockIdx.y];
  const ImgDesc& im = imgs[img];
  const int nr = (im.H >> in.lvl) * (im.W >> in.lvl);
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int r = im.slot_base + im.lvl_off[in.lvl] + i;
  const float a = i < nr ? ul_seed(pl, im, r, i, in) : 0.f;
  const int o = boff[blockIdx.y * gridDim.x + blockIdx.x] + block_excl_scan(a != 0.f ? 1 : 0, buf);
  if (a == 0.f) return;
  const float4 d = pl.d[r];
  const float t = in.t_hist[r];
  samples[o] = make_float4(fmaf(t, d.x, im.c[0]), fmaf(t, d.y, im.c[1]), fmaf(t, d.z, im.c[2]), a);
  sample_lat[o] = im.latent;
  sample_cam[o] = make_int4(img, r, 0, 0);
}

// lam[r] += a grad_p f . v for every sample of the step (grad_p f = the
// residual term's p / (2 |p|) plus the adjoint's per-wave partials).
__global__ void k_ul_lambda(RayPool pl, const float4* samples, const int4* sample_cam, const float* gp_part,
                            const int* n_samples, float* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_samples) return;
  const int4 sc = sample_cam[i];
  if (sc.x < 0) return;
  const float4 smp = samples[i];
  const float rn = sqrtf(smp.x * smp.x + smp.y * smp.y + smp.z * smp.z);
  const float h = rn > 0.f ? 0.5f * smp.w / rn : 0.f;
  float g[3] = {h * smp.x, h * smp.y, h * smp.z};
  const float* pp = gp_part + (size_t)i * 3 * kGpSlots;
  for (int w = 0; w < kGpSlots; ++w) {
    g[0] += pp[3 * w];
    g[1] += pp[3 * w + 1];
    g[2] += pp[3 * w + 2];
  }
  const float4 d = pl.d[sc.y];
  lam[sc.y] += g[0] * d.x + g[1] * d.y + g[2] * d.z;
}

// Coarse-to-fine split in reverse: every ray of level plvl collects the
// adjoints of its four children (fixed order) whose start was its t, i.e. it
// did not miss the sphere and the clamp into the child's interval (computed
// exactly as the forward's split) did not bind.
__global__ __launch_bounds__(256) void k_ul_split(RayPool pl, const ImgDesc* imgs, const int* img_order, int plvl,
                                                  float* lam) {
  const ImgDesc& im = imgs[img_order[blockIdx.y]];
  const int Wp = im.W >> plvl, Hp = im.H >> plvl, Wc = im.W >> (plvl - 1);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= Wp * Hp) return;
  const int pr = im.slot_base + im.lvl_off[plvl] + i;
  if (pl.st[pr] == ST_MISS) return;
  const float tp = pl.d[pr].w;
  const int Vp = i / Wp, Up = i - Vp * Wp;
  float acc = 0.f;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int U = 2 * Up + dx, V = 2 * Vp + dy;
      float3 d;
      float xt, yt, t_lo, t_hi;
      level_ray(im, plvl - 1, U, V, d, xt, yt);
      const bool inside = sphere_interval(im, d, t_lo, t_hi);
      if (inside && tp > t_lo && tp < t_hi) acc += lam[im.slot_base + im.lvl_off[plvl - 1] + V * Wc + U];
    }
  lam[pr] += acc;
}

// Initial adjoints: dL/dd / |(xt, yt, 1)| for level-0 hits (d = t + f, so the
// last t carries the depth gradient directly), 0 for every other ray slot.
__global__ __launch_bounds__(256) void k_ul_init(RayPool pl, const ImgDesc* imgs, const float* g_depth, int spi,
                                                 float* lam) {
  const ImgDesc& im = imgs[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= spi) return;
  const int r = im.slot_base + i;
  float v = 0.f;
  const int pix = i - im.lvl_off[0];
  if (g_depth && pix >= 0 && pix < im.H * im.W && pl.st[r] == ST_HIT) {
    const int V = pix / im.W, U = pix - V * im.W;
    float3 dd;
    float xt, yt;
    level_ray(im, 0, U, V, dd, xt, yt);
    v = g_depth[(size_t)im.out_base + pix] / sqrtf(xt * xt + yt * yt + 1.f);
  }
  lam[r] = v;
}

// ---------------------------------------------------------------------------
// Colour at the hits: the list of hit rays, and the backward's samples (one
// per hit with a nonzero colour gradient: its Eq. 1 point and the gradient).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_color_hits(RayPool pl, const ImgDesc* imgs, int* list, int* counter) {
  const ImgDesc& im = imgs[blockIdx.y];
  const int pix = blockIdx.x * 256 + threadIdx.x;
  const int r = im.slot_base + im.lvl_off[0] + pix;
  const bool hit = pix < im.H * im.W && pl.st[r] == ST_HIT;
  block_append(hit, r, list, counter);
}

__device__ __forceinline__ bool color_sample(const RayPool& pl, const ImgDesc& im, int pix, const float* g) {
  if (pix >= im.H * im.W || pl.st[im.slot_base + im.lvl_off[0] + pix] != ST_HIT) return false;
  const float* gq = g + 3 * ((size_t)im.out_base + pix);
  return gq[0] != 0.f || gq[1] != 0.f || gq[2] != 0.f;
}

__global__ __launch_bounds__(256) void k_color_count(RayPool pl, const ImgDesc* imgs, const int* img_order,
                                                     const float* g_rgb, int* bsum) {
  __shared__ int red[256];
  const ImgDesc& im = imgs[img_order[blockIdx.y]];
  const int pix = blockIdx.x * 256 + threadIdx.x;
  red[threadIdx.x] = color_sample(pl, im, pix, g_rgb) ? 1 : 0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_color_write(RayPool pl, const ImgDesc* imgs, const int* img_order,
                                                     const float* g_rgb, const int* boff, float4* samples,
                                                     float4* cseed, int* sample_lat) {
  __shared__ int buf[256];
  const ImgDesc& im = imgs[img_order[blockIdx.y]];
  const int pix = blockIdx.x * 256 + threadIdx.x;
  const bool take = color_sample(pl, im, pix, g_rgb);
  const int o = boff[blockIdx.y * gridDim.x + blockIdx.x] + block_excl_scan(take ? 1 : 0, buf);
  if (!take) return;
  const int r = im.slot_base + im.lvl_off[0] + pix;
  const float4 d = pl.d[r];
  const float dd = d.w + pl.flast[r];                   // Eq. 1 ray distance
  const float* gq = g_rgb + 3 * ((size_t)im.out_base + pix);
  samples[o] = make_float4(fmaf(dd, d.x, im.c[0]), fmaf(dd, d.y, im.c[1]), fmaf(dd, d.z, im.c[2]), 0.f);
  cseed[o] = make_float4(gq[0], gq[1], gq[2], 0.f);
  sample_lat[o] = im.latent;
}

__global__ void k_fill_f4(float4* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_init_level(const RayPool& pl, ImgDesc* imgs, const int* imgs_list, int n_img, int max_rays, int* list,
                       int* counter, hipStream_t s) {
  if (n_img <= 0 || max_rays <= 0) return;
  hipLaunchKernelGGL(k_init_level, dim3(nblk(max_rays, 256), n_img), dim3(256), 0, s, pl, imgs, imgs_list, list,
                     counter);
}
void launch_split(const RayPool& pl, ImgDesc* imgs, const int* imgs_list, int n_img, int max_children,
                  int child_lvl, int child_step, int* list, int* counter, hipStream_t s, int* counter_tail,
                  int tail_end) {
  if (n_img <= 0 || max_children <= 0) return;
  hipLaunchKernelGGL(k_split, dim3(nblk(max_children, 1024), n_img), dim3(1024), 0, s, pl, imgs, imgs_list,
                     child_lvl, child_step, list, counter, counter_tail, tail_end);
  hipLaunchKernelGGL(k_set_level, dim3(nblk(n_img, 256)), dim3(256), 0, s, imgs, imgs_list, n_img, child_lvl);
}
void launch_finalize(const RayPool& pl, const ImgDesc* imgs, const int* imgs_list, int n_img, int hw,
                     const FinalizeOut& o, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nblk(hw, 1024), n_img), dim3(1024), 0, s, pl, imgs, imgs_list, o);
}
void launch_normals(const RayPool& pl, const ImgDesc* imgs, const int* hits, const int* hit_count, int max_hits,
                    const float* fv, float delta, float* normal, float4* nraw, hipStream_t s) {
  if (max_hits <= 0) return;
  hipLaunchKernelGGL(k_normals, dim3(nblk(max_hits, 256)), dim3(256), 0, s, pl, imgs, hits, hit_count, fv, delta,
                     normal, nraw);
}
void launch_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent, int n_img,
                    int hw, int n_lat, int tile, const SeedIn& in, int* bsum, int* boff, int* seg_base,
                    int* seg_total, int* seg_padded, int* n_samples, float4* samples, int* sample_lat, hipStream_t s,
                    int lat_fixed, const SplitList* sl, int4* sample_cam) {
  const int bpi = (int)nblk(hw, 256);
  const bool split = sl != nullptr && in.hit_pix != nullptr;
  hipLaunchKernelGGL(k_samples_count, dim3(bpi, n_img), dim3(256), 0, s, pl, imgs, img_order, in, bsum,
                     split ? sl->bsum : nullptr);
  hipLaunchKernelGGL(k_samples_scan, dim3(1), dim3(1024), 0, s, bsum, n_img, bpi, img_order, img_latent, lat_fixed,
                     tile, n_lat, boff, seg_base, seg_total, seg_padded, nullptr, n_samples);
  if (split)
    hipLaunchKernelGGL(k_samples_scan, dim3(1), dim3(1024), 0, s, sl->bsum, n_img, bpi, img_order, img_latent,
                       lat_fixed, tile, n_lat, sl->boff, sl->seg_base, sl->seg_total, sl->seg_padded, n_samples,
                       n_samples + 2);
  hipLaunchKernelGGL(k_samples_write, dim3(bpi, n_img), dim3(256), 0, s, pl, imgs, img_order, in, boff,
                     split ? sl->boff : nullptr, samples, sample_lat, split ? sl->sample_idx : nullptr, sample_cam);
  hipLaunchKernelGGL(k_samples_pad, dim3(n_lat), dim3(256), 0, s, seg_base, seg_total, seg_padded, samples,
                     sample_lat, nullptr, sample_cam);
  if (split)
    hipLaunchKernelGGL(k_samples_pad, dim3(n_lat), dim3(256), 0, s, sl->seg_base, sl->seg_total, sl->seg_padded,
                       samples, sample_lat, sl->sample_idx, nullptr);
}
void launch_samples_pad(int n_lat, const int* seg_base, const int* seg_total, const int* seg_padded, float4* samples,
                        int* sample_lat, hipStream_t s) {
  hipLaunchKernelGGL(k_samples_pad, dim3(n_lat), dim3(256), 0, s, seg_base, seg_total, seg_padded, samples,
                     sample_lat, nullptr, nullptr);
}
// grad_p f . v at each hit's Eq. 1 point (unit seeds): the adjoint's per-wave
// partials plus the residual term 0.5 p / |p|; 0 where the ray grazes the
// surface (|grad f . v| <= 1e-2 |grad f|), which then gets no implicit depth term.
__global__ void k_hit_gv(RayPool pl, const ImgDesc* imgs, const float4* samples, const int4* sample_cam,
                         const float* gp_part, const int* n_samples, float* gv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_samples) return;
  const int4 sc = sample_cam[i];
  if (sc.x < 0) return;
  const ImgDesc& im = imgs[sc.x];
  const float4 smp = samples[i];
  const float rn = sqrtf(smp.x * smp.x + smp.y * smp.y + smp.z * smp.z);
  const float h = rn > 0.f ? 0.5f * smp.w / rn : 0.f;
  float g[3] = {h * smp.x, h * smp.y, h * smp.z};
  const float* pp = gp_part + (size_t)i * 3 * kGpSlots;
  for (int w = 0; w < kGpSlots; ++w) {
    g[0] += pp[3 * w];
    g[1] += pp[3 * w + 1];
    g[2] += pp[3 * w + 2];
  }
  const float4 d = pl.d[im.slot_base + im.lvl_off[0] + sc.y];
  const float dv = g[0] * d.x + g[1] * d.y + g[2] * d.z;
  const float gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  gv[(size_t)im.out_base + sc.y] = fabsf(dv) > 1e-2f * gn ? dv : 0.f;
}

void launch_hit_gv(const RayPool& pl, const ImgDesc* imgs, const float4* samples, const int4* sample_cam,
                   const float* gp_part, const int* n_samples, int max_samples, float* gv, hipStream_t s) {
  if (max_samples <= 0) return;
  hipLaunchKernelGGL(k_hit_gv, dim3(nblk(max_samples, 256)), dim3(256), 0, s, pl, imgs, samples, sample_cam, gp_part,
                     n_samples, gv);
}

void launch_cam_reduce(const RayPool& pl, const ImgDesc* imgs, const int* img_view, int n_img, int n_views,
                       const float4* samples, const int4* sample_cam, const float* gp_part, const int* n_samples,
                       const float* g_sil, float* g_cam, hipStream_t s) {
  hipLaunchKernelGGL(k_cam_reduce, dim3(n_views), dim3(256), 0, s, pl, imgs, img_view, n_img, samples, sample_cam,
                     gp_part, n_samples, g_sil, g_cam);
}
void launch_gz_reduce(float* partial, int kmax, int tile, int max_tiles, const int* seg_base,
                      const int* seg_padded, int n_lat, int w0, int mg0, const float* W0z, int ws, int mgs,
                      const float* Wsz, int L, float* gz, hipStream_t s, int lat0, int accumulate) {
  hipLaunchKernelGGL(k_gz_fold, dim3(nblk(max_tiles, kFold), n_lat), dim3(512), 0, s, partial, kmax, tile, seg_base,
                     seg_padded, lat0);
  hipLaunchKernelGGL(k_gz_reduce, dim3(n_lat), dim3(1024), 0, s, partial, kmax, tile, seg_base, seg_padded, w0, mg0,
                     W0z, ws, mgs, Wsz, L, gz, lat0, accumulate);
}
void launch_apply_levels(ImgDesc* imgs, const AdvEntry* table, const int* hdr, int max_entries, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_levels, dim3(nblk(max_entries > 0 ? max_entries : 1, 256)), dim3(256), 0, s, imgs, table,
                     hdr);
}
void launch_advance(const RayPool& pl, const ImgDesc* imgs, const int* in_list, const int* in_count, int* out_list,
                    int* out_count, const AdvEntry* table, const int* hdr, int* img_active, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_old, dim3(grid), dim3(256), 0, s, pl, imgs, in_list, in_count, out_list, out_count,
                     img_active);
  hipLaunchKernelGGL(k_advance_new, dim3(grid), dim3(256), 0, s, pl, imgs, out_list, out_count, table, hdr,
                     img_active);
}
void launch_render_loss(const float* depth, const float* normal, const float* sil, const float* depth_t,
                        const float* normal_t, const float* sil_t, int n_img, int hw, float w_d, float w_s, float w_n,
                        float* loss, float* g_depth, float* g_normal, float* g_sil, hipStream_t s) {
  hipLaunchKernelGGL(k_render_loss, dim3(n_img), dim3(1024), 0, s, depth, normal, sil, depth_t, normal_t, sil_t, hw,
                     w_d, w_s, w_n, loss, g_depth, g_normal, g_sil);
}
void launch_sum_ordered(const float* a, int n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(64), 0, s, a, n, out);
}
void launch_adam(float* z, float* m, float* v, const float* g, int L, float lr, float b1, float b2, float eps, int t,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(L, 256)), dim3(256), 0, s, z, m, v, g, L, lr, b1, b2, eps, t);
}

void launch_ul_init(const RayPool& pl, const ImgDesc* imgs, int n_img, int spi, const float* g_depth, float* lam,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_ul_init, dim3(nblk(spi, 256), n_img), dim3(256), 0, s, pl, imgs, g_depth, spi, lam);
}
void launch_ul_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent,
                       int n_img, int nr, int n_lat, int tile, const UlIn& in, int* bsum, int* boff, int* seg_base,
                       int* seg_total, int* seg_padded, int* n_samples, float4* samples, int* sample_lat,
                       int4* sample_cam, hipStream_t s) {
  const int bpl = (int)nblk(nr, 256);
  hipLaunchKernelGGL(k_ul_count, dim3(bpl, n_img), dim3(256), 0, s, pl, imgs, img_order, in, bsum);
  hipLaunchKernelGGL(k_samples_scan, dim3(1), dim3(1024), 0, s, bsum, n_img, bpl, img_order, img_latent, 0, tile,
                     n_lat, boff, seg_base, seg_total, seg_padded, nullptr, n_samples);
  hipLaunchKernelGGL(k_ul_write, dim3(bpl, n_img), dim3(256), 0, s, pl, imgs, img_order, in, boff, samples,
                     sample_lat, sample_cam);
  hipLaunchKernelGGL(k_samples_pad, dim3(n_lat), dim3(256), 0, s, seg_base, seg_total, seg_padded, samples,
                     sample_lat, nullptr, sample_cam);
}
void launch_ul_lambda(const RayPool& pl, const float4* samples, const int4* sample_cam, const float* gp_part,
                      const int* n_samples, int max_samples, float* lam, hipStream_t s) {
  if (max_samples <= 0) return;
  hipLaunchKernelGGL(k_ul_lambda, dim3(nblk(max_samples, 256)), dim3(256), 0, s, pl, samples, sample_cam, gp_part,
                     n_samples, lam);
}
void launch_ul_split(const RayPool& pl, const ImgDesc* imgs, const int* img_order, int n_img, int max_parents,
                     int plvl, float* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_ul_split, dim3(nblk(max_parents, 256), n_img), dim3(256), 0, s, pl, imgs, img_order, plvl,
                     lam);
}
void launch_color_hits(const RayPool& pl, const ImgDesc* imgs, int n_img, int hw, int* list, int* counter,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_color_hits, dim3(nblk(hw, 256), n_img), dim3(256), 0, s, pl, imgs, list, counter);
}
void launch_color_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent,
                          int n_img, int hw, int n_lat, int tile, const float* g_rgb, int* bsum, int* boff,
                          int* seg_base, int* seg_total, int* seg_padded, int* n_samples, float4* samples,
                          float4* cseed, int* sample_lat, long long cap, hipStream_t s) {
  const int bpi = (int)nblk(hw, 256);
  hipLaunchKernelGGL(k_fill_f4, dim3(256), dim3(256), 0, s, cseed, cap);
  hipLaunchKernelGGL(k_color_count, dim3(bpi, n_img), dim3(256), 0, s, pl, imgs, img_order, g_rgb, bsum);
  hipLaunchKernelGGL(k_samples_scan, dim3(1), dim3(1024), 0, s, bsum, n_img, bpi, img_order, img_latent, 0, tile,
                     n_lat, boff, seg_base, seg_total, seg_padded, nullptr, n_samples);
  hipLaunchKernelGGL(k_color_write, dim3(bpi, n_img), dim3(256), 0, s, pl, imgs, img_order, g_rgb, boff, samples,
                     cseed, sample_lat);
  hipLaunchKernelGGL(k_samples_pad, dim3(n_lat), dim3(256), 0, s, seg_base, seg_total, seg_padded, samples,
                     sample_lat, nullptr, nullptr);
}
void launch_fill_i32(int* p, int v, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
}
void launch_fill_u64(unsigned long long* p, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
}

}  // namespace dist
