// Launch interface of the celmi kernels (internal).
#pragma once
#include "device.h"

namespace celmi {

struct PrepArgs {
  const double* theta;         // [S*32]
  const double* theta_trial;   // [S*32] used by the trial variant (may be null)
  double fd_step;
  int32_t variant0;            // variant of blockIdx.y == 0
  const int32_t* patch_list;   // patches to prepare (null = patch_offset + blockIdx.x)
  int32_t patch_offset;
  const DPatch* patches;
  const cel_image* images;
  const DProfiles* prof;
  void* tables;                // Table<T>[variants][n_patches]
  int32_t n_patches;
  const uint8_t* active;       // per source (null = all)
  int32_t trial_variant;       // variant evaluated at theta_trial
  int32_t fd;                  // variants 1..54 are central-difference points
  const double* sky_min;       // per patch: smallest sky value (component cut)
  int64_t theta_vstride;       // > 0: variant v reads theta + v * theta_vstride (per-variant points)
  const double* patch_psf;     // [P][kMaxPsf][6] per-patch PSF mixtures (null: the image's)
  int32_t records;             // extra table records: kRecHessian (gt), kRecRuns (rq)
  const uint8_t* active_v;     // per (launch variant, source), row stride active_v_stride (null = all)
  int64_t active_v_stride;
};
constexpr int kRecHessian = 1;
constexpr int kRecRuns = 2;

struct FinalizeArgs {
  int32_t n_jobs;              // sources handled by this launch
  const int32_t* job_src;      // job -> source (null: source = job + src_offset)
  int32_t src_offset;
  int32_t variant0;
  const uint8_t* active;
  const double* theta;
  const double* theta_trial;
  double fd_step;
  const double* slots;
  int64_t slot_variant_stride;
  const int32_t* patch_ptr;    // [S+1]
  const DPatch* patches;
  const double* pix_const;     // [P][2]
  const cel_image* images;
  const DPrior* prior;
  int32_t want_grad;
  double* local;               // [variants][S] (null = not written)
  double* own;                 // [variants][S]
  double* grad;                // [variants][S][32]
  int64_t out_variant_stride;  // = S
  int32_t trial_variant;
  int32_t fd;
  int32_t* err;                // device condition word (CEL_DEVERR_*), may be null
  int64_t theta_vstride;       // as in PrepArgs
  int32_t no_kl;               // 1: the pixel sum alone (point likelihood), no KL
  const uint8_t* active_v;     // per (launch variant, source), row stride active_v_stride (null = all)
  int64_t active_v_stride;
};

template <typename T>
hipError_t launch_prep_tables(const PrepArgs& a, int n_patches_launch, int n_variants, hipStream_t st);
template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int nexp, int ndev, int ppl, bool grad, int n_items,
                        int n_variants, hipStream_t st);
template <typename T>
hipError_t launch_maps(const MapArgs& a, int nexp, int ndev, int ppl, int n_items, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs& a, int n_variants, hipStream_t st);
hipError_t launch_total(const double* own, int n, double* out, hipStream_t st);
hipError_t launch_pixels(const DPatch* patches, const cel_image* images, const double* knots, const float* pixels,
                         const int64_t* user_off, float2* xs, double2* xs64, int n_patches, hipStream_t st);
// unconstrained parameters [n][32] that make the objective's pixel terms the exact Poisson
// log-likelihood at point values z [n][CEL_Z_N] (type probability 0 or 1, zero variances);
// ok[n] (may be null) records which rows lie in the support
hipError_t launch_point_theta(const double* z, int64_t n, double* theta, uint8_t* ok, hipStream_t st);
// log p(w | a) of n point values z [n][CEL_Z_N] under the plan's prior tables
hipError_t launch_log_prior(const DPrior* prior, const double* z, int64_t n, double* out, hipStream_t st);
// ll[i] = -infinity where ok[i] == 0 and source i % S is selected (mask[S])
hipError_t launch_support_masked(const uint8_t* ok, const uint8_t* mask, int S, int64_t n, double* ll, hipStream_t st);
// data constants x log x - x - log x! of the counts 0 .. kCountTable - 1 (once per context)
constexpr int kCountTable = 4096;
hipError_t launch_count_table(double* table, hipStream_t st);
hipError_t launch_pixconst(const DPatch* patches, const int32_t* nbr_idx, const float2* xs, const double* table,
                           double* out, double* sky_min, int n_patches, hipStream_t st);

}  // namespace celmi
