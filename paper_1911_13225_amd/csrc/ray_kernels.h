// Launchers of the ray bookkeeping kernels (ray_kernels.hip).
#pragma once
#include "dist_internal.h"

namespace dist {

struct FinalizeOut {
  float* depth;
  float* dist;
  float* sil;
  float* normal;
  uint8_t* status;
  uint8_t* nsteps;
  float4* nraw;      // per pixel (nx, ny, nz, |n|), zeroed here, filled by the normal pass
  int* hits;
  int* hit_count;
  int want_hits;
  int* hit_pix;      // per output pixel: its index in hits, -1 if none (or null)
};

// One image that starts rays this tick: split into level `lvl` (split = 1) or
// (re)started at its coarsest level `lvl` (split = 0); its new rays occupy
// positions [begin, begin + count) of the tick's new-ray range.
struct AdvEntry {
  int img, lvl, step, split, begin, count;
};

struct SeedIn {
  const float* g_depth;
  const float* g_normal;
  const float* g_sil;
  const float4* nraw;
  float delta;
  const int* hit_pix;  // split layout: per output pixel, its index in the forward's hit list
  // exact depth gradient: 1 = only one unit-seed sample per hit with a depth
  // gradient, at its Eq. 1 point (to measure grad f . v there); with imp_gv
  // the depth term of a hit is one sample at that point with seed
  // -dL/dz_c / |(xt, yt, 1)| / (grad f . v) (imp_gv[q] = 0: no depth term)
  int hit_mode;
  const float* imp_gv;
};

// One step of the gradient through the unrolled march: the rays of level lvl
// that took global step `step`, their t at that step (t_hist, indexed by ray
// slot) and the current adjoints of t (lam, by ray slot).
struct UlIn {
  int step, lvl;
  const float* g_depth;
  const float* g_sil;
  const float* t_hist;
  const float* lam;
};

// Second sample list of the split layout (normal-stencil samples).
struct SplitList {
  int* bsum;
  int* boff;
  int* seg_base;
  int* seg_total;
  int* seg_padded;
  int* sample_idx;
};

void launch_init_level(const RayPool& pl, ImgDesc* imgs, const int* imgs_list, int n_img, int max_rays, int* list,
                       int* counter, hipStream_t s);
void launch_split(const RayPool& pl, ImgDesc* imgs, const int* imgs_list, int n_img, int max_children,
                  int child_lvl, int child_step, int* list, int* counter, hipStream_t s,
                  int* counter_tail = nullptr, int tail_end = 0);
void launch_finalize(const RayPool& pl, const ImgDesc* imgs, const int* imgs_list, int n_img, int hw,
                     const FinalizeOut& o, hipStream_t s);
void launch_normals(const RayPool& pl, const ImgDesc* imgs, const int* hits, const int* hit_count, int max_hits,
                    const float* fv, float delta, float* normal, float4* nraw, hipStream_t s);
void launch_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent, int n_img,
                    int hw, int n_lat, int tile, const SeedIn& in, int* bsum, int* boff, int* seg_base,
                    int* seg_total, int* seg_padded, int* n_samples, float4* samples, int* sample_lat, hipStream_t s,
                    int lat_fixed = 0, const SplitList* split = nullptr, int4* sample_cam = nullptr);
void launch_samples_pad(int n_lat, const int* seg_base, const int* seg_total, const int* seg_padded, float4* samples,
                        int* sample_lat, hipStream_t s);
void launch_gz_reduce(float* partial, int kmax, int tile, int max_tiles, const int* seg_base,
                      const int* seg_padded, int n_lat, int w0, int mg0, const float* W0z, int ws, int mgs,
                      const float* Wsz, int L, float* gz, hipStream_t s, int lat0 = 0, int accumulate = 0);
void launch_cam_reduce(const RayPool& pl, const ImgDesc* imgs, const int* img_view, int n_img, int n_views,
                       const float4* samples, const int4* sample_cam, const float* gp_part, const int* n_samples,
                       const float* g_sil, float* g_cam, hipStream_t s);
void launch_hit_gv(const RayPool& pl, const ImgDesc* imgs, const float4* samples, const int4* sample_cam,
                   const float* gp_part, const int* n_samples, int max_samples, float* gv, hipStream_t s);
void launch_ul_init(const RayPool& pl, const ImgDesc* imgs, int n_img, int spi, const float* g_depth, float* lam,
                    hipStream_t s);
void launch_ul_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent,
                       int n_img, int nr, int n_lat, int tile, const UlIn& in, int* bsum, int* boff, int* seg_base,
                       int* seg_total, int* seg_padded, int* n_samples, float4* samples, int* sample_lat,
                       int4* sample_cam, hipStream_t s);
void launch_ul_lambda(const RayPool& pl, const float4* samples, const int4* sample_cam, const float* gp_part,
                      const int* n_samples, int max_samples, float* lam, hipStream_t s);
void launch_ul_split(const RayPool& pl, const ImgDesc* imgs, const int* img_order, int n_img, int max_parents,
                     int plvl, float* lam, hipStream_t s);
void launch_color_hits(const RayPool& pl, const ImgDesc* imgs, int n_img, int hw, int* list, int* counter,
                       hipStream_t s);
void launch_color_samples(const RayPool& pl, const ImgDesc* imgs, const int* img_order, const int* img_latent,
                          int n_img, int hw, int n_lat, int tile, const float* g_rgb, int* bsum, int* boff,
                          int* seg_base, int* seg_total, int* seg_padded, int* n_samples, float4* samples,
                          float4* cseed, int* sample_lat, long long cap, hipStream_t s);
void launch_apply_levels(ImgDesc* imgs, const AdvEntry* table, const int* hdr, int max_entries, hipStream_t s);
// Two launches: the previous list's survivors, then the rays that start this
// tick (split children and (re)started images).
void launch_advance(const RayPool& pl, const ImgDesc* imgs, const int* in_list, const int* in_count, int* out_list,
                    int* out_count, const AdvEntry* table, const int* hdr, int* img_active, int grid, hipStream_t s);
// Per-image loss of inverse optimisation (L1 depth, silhouette hinge, normal
// term) and its map gradients; one workgroup per image, fixed order.
void launch_render_loss(const float* depth, const float* normal, const float* sil, const float* depth_t,
                        const float* normal_t, const float* sil_t, int n_img, int hw, float w_d, float w_s, float w_n,
                        float* loss, float* g_depth, float* g_normal, float* g_sil, hipStream_t s);
void launch_sum_ordered(const float* a, int n, float* out, hipStream_t s);
void launch_adam(float* z, float* m, float* v, const float* g, int L, float lr, float b1, float b2, float eps, int t,
                 hipStream_t s);
void launch_fill_i32(int* p, int v, int n, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int n, hipStream_t s);

}  // namespace dist
