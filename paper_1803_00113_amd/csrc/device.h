// Internal device-side layouts of the celmi library (gfx950).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/celmi.h"

namespace celmi {

constexpr int kThetaN = CEL_N_THETA;
constexpr int kParamN = CEL_N_PARAM;
constexpr int kMaxPsf = CEL_MAX_PSF;
constexpr int kMaxProf = CEL_MAX_PROFILE;
constexpr int kSlots = 16;          // fp64 partial sums per work item (13 used)
constexpr int kVariants = 56;       // 0 base, 1..27 +h, 28..54 -h, 55 trial point
constexpr int kWave = 64;

// slot indices of the per-(work item) partial sums
enum Slot {
  S_CE_F0 = 0,   // sum c_E f0
  S_CE_F1,       // sum c_E f1
  S_CV_F00,      // sum c_V f0^2
  S_CV_F11,      // sum c_V f1^2
  S_CV_F01,      // sum c_V f0 f1
  S_MU_X,        // sum rho0 df0/dmu_x + rho1 df1/dmu_x
  S_MU_Y,
  S_S_XX,        // sum rho0 df0/dS_xx  (S = pixel-frame galaxy covariance)
  S_S_XY,        // sum rho0 df0/dS_xy  (symmetric: both off-diagonal entries)
  S_S_YY,
  S_PI,          // sum rho0 df0/de_profile
  S_T,           // sum of the centred pixel term over the work item
  S_T_OWN,       // same, pixels owned by this source only
};

// Per (variant, patch) table of mixture components in patch-local pixel coordinates.
// hdr: L0, L1, w0, w1, k0, k1, w01, pi  (E_s = w0 L0 f0 + w1 L1 f1,
//      V_s = k0 f0^2 + k1 f1^2 + w01 (L0 f0 - L1 f1)^2, f0 = pi f_dev + (1 - pi) f_exp)
// star[k]: mean_x, mean_y, P_xx, P_xy, P_yy, log2 weight (weight includes the normaliser)
// gal[k][j]: P_xx, P_xy, P_yy, log2 weight  (j < n_exp: exponential, then de Vaucouleurs)
// rc2s[k], rc2[k][j]: squared distance from the component's centre beyond which flux times
// density stays below 2^-30 (float tables) or 2^-60 (double) of the patch's smallest sky
// value (bounded through the covariance's largest eigenvalue); -1 = negligible everywhere
// hdr[8..9]: e0, e1 = expm1(variance of log l given the type) (for the analytic Hessian)
// gt[k][j]: tau, tau^2, then tau^2/2 tr(E1 P E2 P) for the S-parameter pairs (xx,xx),
//           (xx,xy), (xx,yy), (xy,xy), (xy,yy), (yy,yy)
// hdr[10..11]: the source centre mu in patch-local pixels
// sq[k], gq[k][j]: (-log2(e)/2 (P_xx, P_xy, P_yy), log2 weight) -- the exponent of a
//   component at offset d from its centre is q0 dx^2 + q1 (2 dx dy) + q2 dy^2 + q3
//   (values-only evaluation: neighbour maps, Hessian)
// rq[k][0], rq[k][1 + j]: exp(-P_xx) of the star and of galaxy component j = 2^(2 q0), the
//   factor by which the ratio of a component's values at consecutive columns changes
//   (values along a row by recurrence: neighbour maps; written when that map variant is on)
// gq[k][j][4..7]: (c^2 P_xx, c^2 P_xy, c^2 P_yy, tau/2), c = -log2(e)/2 -- with u' = c P d
//   (from gq[k][j][0..2]) the own-source kernel forms the exponent as d . u' + q3 and the
//   covariance derivative from u' u'^T - c^2 P = c^2 (u u^T - P); its mean and covariance
//   sums are c and c^2 times the plain ones and are divided back once per slot row.  One
//   component's eight values are 32 bytes, copied to LDS once per work item.
// gal and gt are written only for the exact Hessian's preparations
template <typename T>
// The records the pixel kernels read for every component (header, star records, cut radii,
// exponent records) come first and together, so that a wavefront's scalar loads of one
// patch's table touch as few cache lines as possible; the Hessian's and the other kernels'
// records follow.  gq starts on a 32-byte boundary (one 32-byte load per component) and
// the table's size is a multiple of 64 bytes.
struct alignas(64) Table {
  T hdr[16];
  T star[kMaxPsf][8];
  T rc2s[kMaxPsf];
  T rc2[kMaxPsf][2 * kMaxProf];
  T sq[kMaxPsf][4];
  T pad0[4];
  T gq[kMaxPsf][2 * kMaxProf][8];
  T gal[kMaxPsf][2 * kMaxProf][4];
  T gt[kMaxPsf][2 * kMaxProf][8];
  T rq[kMaxPsf][1 + 2 * kMaxProf];
  T pad1[20];
};

// the exponent's scale in the own-source records: c = -log2(e) / 2
constexpr double kExpScale = -0.72134752044448170368;

struct DPatch {
  int32_t src, img, x0, y0, w, h;
  int64_t off;            // into the (count, sky) pixel array
  int32_t nbr_begin, nbr_end;   // into nbr_idx: other sources' patches intersecting this one
  int32_t task_begin, task_end; // work items of this patch (patch-major order)
};

struct DTask {
  int32_t patch, pix_begin, pix_end, pad;
};

struct DPrior {
  double logit_a, log_a, log_1ma;
  double r[2][2];
  double c_logw[2][CEL_N_COLOUR_COMPONENTS];
  double c_mean[2][CEL_N_COLOUR_COMPONENTS][4];
  double c_prec[2][CEL_N_COLOUR_COMPONENTS][4][4];
  double c_logdet[2][CEL_N_COLOUR_COMPONENTS];
  double radius[2];
  double profile[2], axis[2];
  double lbeta_profile, lbeta_axis;
};

struct DProfiles {
  int32_t n_exp, n_dev;
  double alpha[2 * kMaxProf], tau[2 * kMaxProf];   // exp first, then dev
};

// Arguments of the pixel kernel.
template <typename T>
struct FusedArgs {
  const DTask* tasks;
  const int32_t* order;        // launch order -> task id (nullptr = identity)
  int32_t order_offset;        // first entry of `order` (or task id) for this launch
  const DPatch* patches;
  const int32_t* nbr_idx;
  const Table<T>* base;        // variant-0 tables [P]
  const Table<T>* own;         // tables of the variant being evaluated, [P] per variant
  int64_t variant_stride;      // tables per variant (= P)
  const void* xs;              // (count, sky) per packed pixel: float2 (T=float) or double2
  const void* maps;            // (E_s, V_s) of each patch's own source per packed pixel
  double* slots;               // [variant][n_tasks][kSlots]
  int64_t slot_variant_stride; // = n_tasks * kSlots
  const uint8_t* active;       // per source (nullptr = all)
  int32_t variant0;            // variant index of blockIdx.y == 0
  const int32_t* img_npsf;     // PSF components per image
  const uint8_t* active_v;     // per (launch variant, source), row stride active_v_stride (nullptr = all)
  int64_t active_v_stride;
  double unscale[2];           // set by the launcher: 1/c and 1/c^2 for the centre and covariance sums
};

// A work item of the moment-map pass: pixels [pix_begin, pix_end) of a patch's overlap box
// (the bounding box of its intersections with the other sources' patches, w pixels wide,
// at patch-local (x0, y0)), row-major within the box.  Neighbours read a patch's moments
// only inside that box.
struct DMapTask {
  int32_t patch, pix_begin, pix_end, x0, y0, w, pad0, pad1;
};

struct MapArgs {
  const DMapTask* tasks;       // in launch order
  const DPatch* patches;
  const void* base;            // variant-0 tables
  void* maps;                  // out: (E_s, V_s) per packed pixel
  const int32_t* img_npsf;
};

}  // namespace celmi
