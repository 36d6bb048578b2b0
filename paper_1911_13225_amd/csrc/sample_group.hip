// Grouping of explicit decoder samples by latent code, on the device, for
// the VJP entry point (the per-sample term of Eq. 2 summed per latent).  The
// recompute-and-VJP kernel takes tiles that each hold samples of one latent,
// so the samples are reordered into per-latent segments padded to whole
// tiles: a stable radix sort of (latent id, sample index) pairs keeps the
// samples of a latent in index order, so the tiles, their column sums and
// the per-latent reduction see the samples in a fixed order and the result
// is reproducible bit for bit.
#include <hipcub/hipcub.hpp>

#include "dist_internal.h"

namespace dist {

__global__ void k_group_zero(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// keys = latent ids clamped to [0, n_lat) (as the plain decoder query does),
// values = sample indices; counts per latent (integer atomics: exact)
__global__ void k_group_keys(const int32_t* __restrict__ lat, int n_lat, int n, int* __restrict__ keys,
                             int* __restrict__ vals, int* __restrict__ cnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int l = min(max((int)lat[i], 0), n_lat - 1);
    keys[i] = l;
    vals[i] = i;
    atomicAdd(&cnt[l], 1);
  }
}

// per latent: samples and the segment length padded to whole tiles
__global__ void k_group_pad(const int* __restrict__ cnt, int n_lat, int tile, int* __restrict__ total,
                            int* __restrict__ padded) {
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_lat; l += gridDim.x * blockDim.x) {
    const int c = cnt[l];
    total[l] = c;
    padded[l] = (c + tile - 1) / tile * tile;
  }
}

__global__ void k_group_count(const int* __restrict__ base, const int* __restrict__ padded, int n_lat,
                              int* __restrict__ n_samples) {
  if (blockIdx.x == 0 && threadIdx.x == 0) n_samples[0] = base[n_lat - 1] + padded[n_lat - 1];
}

// sorted position s -> slot base[l] + (s - start[l]) of its latent's segment
__global__ void k_group_gather(const int* __restrict__ keys, const int* __restrict__ vals,
                               const int* __restrict__ start, const int* __restrict__ base,
                               const float* __restrict__ pts, const float* __restrict__ seeds, int n,
                               float4* __restrict__ samples, int* __restrict__ sample_lat) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const int l = keys[s], i = vals[s];
    const int o = base[l] + (s - start[l]);
    samples[o] = make_float4(pts[3 * (size_t)i], pts[3 * (size_t)i + 1], pts[3 * (size_t)i + 2], seeds[i]);
    sample_lat[o] = l;
  }
}

// the padding slots of every segment: zero seed (no contribution), the
// segment's latent
__global__ void k_group_fill(const int* __restrict__ cnt, const int* __restrict__ padded,
                             const int* __restrict__ base, int n_lat, int tile, float4* __restrict__ samples,
                             int* __restrict__ sample_lat) {
  const long long total = (long long)n_lat * tile;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(t / tile), k = cnt[l] + (int)(t % tile);
    if (k < padded[l]) {
      samples[base[l] + k] = make_float4(0.f, 0.f, 0.f, 0.f);
      sample_lat[base[l] + k] = l;
    }
  }
}

static int key_bits(int n_lat) {
  int b = 1;
  while ((1LL << b) < n_lat) ++b;
  return b;
}

size_t group_temp_bytes(int n, int n_lat) {
  size_t a = 0, b = 0;
  const int m = n > 0 ? n : 1;
  // a failed size query leaves its size at 0: the sort or scan then reports
  // the short temporary buffer as an error, which group_samples returns
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const int*)nullptr, (int*)nullptr, (const int*)nullptr,
                                         (int*)nullptr, m, 0, key_bits(n_lat)) != hipSuccess)
    a = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int*)nullptr, (int*)nullptr, n_lat) != hipSuccess) b = 0;
  return std::max(a, b) + 256;
}

static int grid_for(long long work) { return (int)std::max<long long>(1, std::min<long long>((work + 255) / 256, 4096)); }

hipError_t group_samples(const GroupArgs& g, hipStream_t st) {
  const int L = g.n_lat;
  hipLaunchKernelGGL(k_group_zero, dim3(grid_for(L)), dim3(256), 0, st, g.cnt, L);
  if (g.n > 0) {
    hipLaunchKernelGGL(k_group_keys, dim3(grid_for(g.n)), dim3(256), 0, st, g.lat, L, g.n, g.keys_in, g.vals_in,
                       g.cnt);
    size_t tb = g.temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(g.temp, tb, g.keys_in, g.keys_out, g.vals_in, g.vals_out, g.n,
                                                      0, key_bits(L), st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_group_pad, dim3(grid_for(L)), dim3(256), 0, st, g.cnt, L, g.tile, g.seg_total, g.seg_padded);
  size_t tb = g.temp_bytes;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(g.temp, tb, g.seg_padded, g.seg_base, L, st);
  if (e != hipSuccess) return e;
  tb = g.temp_bytes;
  e = hipcub::DeviceScan::ExclusiveSum(g.temp, tb, g.cnt, g.start, L, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_count, dim3(1), dim3(64), 0, st, g.seg_base, g.seg_padded, L, g.n_samples);
  if (g.n > 0)
    hipLaunchKernelGGL(k_group_gather, dim3(grid_for(g.n)), dim3(256), 0, st, g.keys_out, g.vals_out, g.start,
                       g.seg_base, g.pts, g.seeds, g.n, g.samples, g.sample_lat);
  hipLaunchKernelGGL(k_group_fill, dim3(grid_for((long long)L * g.tile)), dim3(256), 0, st, g.cnt, g.seg_padded,
                     g.seg_base, L, g.tile, g.samples, g.sample_lat);
  return hipGetLastError();
}

}  // namespace dist
