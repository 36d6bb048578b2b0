// Cross-view photometric loss of multi-view reconstruction (paper Sec. 4,
// "multi-view" objective; App. C, depth/normal/silhouette/color loss): every
// rendered pixel of view i is lifted to its surface point with the rendered
// depth, projected into a neighbouring view j, and compared (L1) with view j's
// colour there (bilinear); the gradient flows to the depth of view i.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ctx.h"

namespace dist {

constexpr int kPhotoViews = 16, kPhotoPairs = 64;
constexpr float kPhotoVis = 1e-3f;      // Delta_d^2 below this: visible in both views

struct PhotoCam {
  float fx, fy, cx, cy;
  float R[9];                            // camera-to-world, row-major
  float c[3];
};

struct PhotoArgs {
  PhotoCam cam[kPhotoViews];
  int2 pair[kPhotoPairs];                // (i, j): warp view j into view i
  int n_pairs, H, W;
  float scale;                           // weight / (H W)
  const float* depth;                    // [n][H][W] z_c, inf = background
  const float* images;                   // [n][H][W][3]
  float* loss_map;                       // [n][H][W]
  float* g_depth;                        // [n][H][W] or null
};

__device__ __forceinline__ float bil(const float* I, int W, int a0, int b0, float al, float be, int ch, float& da,
                                     float& db) {
  const float i00 = I[((size_t)b0 * W + a0) * 3 + ch], i01 = I[((size_t)b0 * W + a0 + 1) * 3 + ch];
  const float i10 = I[((size_t)(b0 + 1) * W + a0) * 3 + ch], i11 = I[((size_t)(b0 + 1) * W + a0 + 1) * 3 + ch];
  da = (1.f - be) * (i01 - i00) + be * (i11 - i10);
  db = (1.f - al) * (i10 - i00) + al * (i11 - i01);
  return (1.f - be) * ((1.f - al) * i00 + al * i01) + be * ((1.f - al) * i10 + al * i11);
}

// One thread per pixel of view blockIdx.y; the pairs whose first view it is
// are visited in list order, so each pixel's loss and gradient are written
// once (no atomics, bitwise reproducible).
__global__ __launch_bounds__(256) void k_photo(PhotoArgs a) {
  const int i = blockIdx.y;
  const int hw = a.H * a.W;
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= hw) return;
  const size_t q = (size_t)i * hw + x;
  const float z = a.depth[q];
  float lsum = 0.f, gsum = 0.f;
  if (z != INFINITY && z == z) {
    const PhotoCam& ci = a.cam[i];
    const int v = x / a.W, u = x - v * a.W;
    // the pixel's ray (Sec. 3.3): direction R K^-1 (u + 1/2, v + 1/2, 1), normalised
    const float xt = ((float)u + 0.5f - ci.cx) / ci.fx, yt = ((float)v + 0.5f - ci.cy) / ci.fy;
    const float nrm = sqrtf(xt * xt + yt * yt + 1.f);
    const float dc[3] = {xt / nrm, yt / nrm, 1.f / nrm};
    float dir[3], X[3];
    for (int r = 0; r < 3; ++r) {
      dir[r] = ci.R[3 * r] * dc[0] + ci.R[3 * r + 1] * dc[1] + ci.R[3 * r + 2] * dc[2];
      X[r] = ci.c[r] + z * nrm * dir[r];
    }
    const float* Ii = a.images + q * 3;
    for (int p = 0; p < a.n_pairs; ++p) {
      if (a.pair[p].x != i) continue;
      const int j = a.pair[p].y;
      const PhotoCam& cj = a.cam[j];
      // camera frame of view j: R^T (X - c); and its derivative along the ray of view i
      float Xc[3], dX[3];
      for (int k = 0; k < 3; ++k) {
        Xc[k] = cj.R[k] * (X[0] - cj.c[0]) + cj.R[3 + k] * (X[1] - cj.c[1]) + cj.R[6 + k] * (X[2] - cj.c[2]);
        dX[k] = nrm * (cj.R[k] * dir[0] + cj.R[3 + k] * dir[1] + cj.R[6 + k] * dir[2]);
      }
      if (!(Xc[2] > 0.f)) continue;
      const float fa = cj.fx * Xc[0] / Xc[2] + cj.cx - 0.5f;     // pixel-index coordinates in view j
      const float fb = cj.fy * Xc[1] / Xc[2] + cj.cy - 0.5f;
      const float fan = floorf(fa + 0.5f), fbn = floorf(fb + 0.5f), fa0 = floorf(fa), fb0 = floorf(fb);
      // range checks in float before any conversion to int
      if (!(fan >= 0.f && fan < (float)a.W && fbn >= 0.f && fbn < (float)a.H)) continue;
      if (!(fa0 >= 0.f && fa0 + 1.f < (float)a.W && fb0 >= 0.f && fb0 + 1.f < (float)a.H)) continue;
      const int an = (int)fan, bn = (int)fbn, a0 = (int)fa0, b0 = (int)fb0;
      const float dj = a.depth[(size_t)j * hw + (size_t)bn * a.W + an];
      if (!(dj != INFINITY && dj == dj)) continue;
      const float dd = Xc[2] - dj;
      if (!(dd * dd < kPhotoVis)) continue;
      const float al = fa - fa0, be = fb - fb0;
      const float iz = 1.f / Xc[2];
      const float da = cj.fx * (dX[0] * iz - Xc[0] * dX[2] * iz * iz);
      const float db = cj.fy * (dX[1] * iz - Xc[1] * dX[2] * iz * iz);
      const float* Ij = a.images + (size_t)j * hw * 3;
      for (int ch = 0; ch < 3; ++ch) {
        float ga, gb;
        const float w = bil(Ij, a.W, a0, b0, al, be, ch, ga, gb);
        const float r = Ii[ch] - w;
        lsum += fabsf(r);
        const float sg = r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f);
        gsum -= sg * (ga * da + gb * db);
      }
    }
  }
  a.loss_map[q] = a.scale * lsum;
  if (a.g_depth) a.g_depth[q] = a.scale * gsum;
}

// Sum of the loss map in a fixed order (one workgroup).
__global__ __launch_bounds__(1024) void k_photo_sum(const float* m, long long n, float* out) {
  __shared__ float red[1024];
  float s = 0.f;
  for (long long k = threadIdx.x; k < n; k += 1024) s += m[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace dist

using namespace dist;

extern "C" int dist_photometric_loss(const dist_camera* cams, int32_t n_views, const float* depth,
                                     const float* images, const int32_t* pairs, int32_t n_pairs, float weight,
                                     float* loss_map, float* loss, float* g_depth, void* stream) {
  if (!cams || !depth || !images || !pairs || !loss_map || !loss) return dist_set_error(DIST_EINVAL, "null argument");
  if (n_views < 1 || n_views > kPhotoViews) return dist_set_error(DIST_EINVAL, "n_views must be in [1, 16]");
  if (n_pairs < 1 || n_pairs > kPhotoPairs) return dist_set_error(DIST_EINVAL, "n_pairs must be in [1, 64]");
  if (!std::isfinite(weight)) return dist_set_error(DIST_EINVAL, "weight must be finite");
  const int H = cams[0].H, W = cams[0].W;
  if (H < 2 || W < 2 || (long long)H * W > (1 << 22))
    return dist_set_error(DIST_EINVAL, "H and W must be at least 2 (at most 4M pixels)");
  PhotoArgs a{};
  for (int v = 0; v < n_views; ++v) {
    if (cams[v].H != H || cams[v].W != W) return dist_set_error(DIST_EINVAL, "all views must share H and W");
    if (!(cams[v].fx != 0.f) || !(cams[v].fy != 0.f)) return dist_set_error(DIST_EINVAL, "zero focal length");
    PhotoCam& c = a.cam[v];
    c.fx = cams[v].fx;
    c.fy = cams[v].fy;
    c.cx = cams[v].cx;
    c.cy = cams[v].cy;
    for (int k = 0; k < 9; ++k) c.R[k] = cams[v].R_wc[k];
    for (int k = 0; k < 3; ++k) c.c[k] = cams[v].c[k];
  }
  for (int p = 0; p < n_pairs; ++p) {
    const int i = pairs[2 * p], j = pairs[2 * p + 1];
    if (i < 0 || i >= n_views || j < 0 || j >= n_views) return dist_set_error(DIST_EINVAL, "pair %d out of range", p);
    a.pair[p] = make_int2(i, j);
  }
  a.n_pairs = n_pairs;
  a.H = H;
  a.W = W;
  a.scale = weight / (float)(H * W);
  a.depth = depth;
  a.images = images;
  a.loss_map = loss_map;
  a.g_depth = g_depth;
  hipStream_t st = (hipStream_t)stream;
  const int hw = H * W;
  hipLaunchKernelGGL(k_photo, dim3((hw + 255) / 256, n_views), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_photo_sum, dim3(1), dim3(1024), 0, st, loss_map, (long long)n_views * hw, loss);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dist_set_error(DIST_EHIP, "photometric loss launch failed: %s", hipGetErrorString(e));
  return DIST_OK;
}
