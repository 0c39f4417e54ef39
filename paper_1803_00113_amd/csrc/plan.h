// Plan and context structures (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <vector>

#include "device.h"

// Pinned host words, event and stream of a plan's Newton calls (reused across plans).
struct HostKit {
  uint8_t* h_mask = nullptr;
  size_t mask_cap = 0;
  int32_t* h_lists = nullptr;     // a Newton step's source, patch and work-item lists
  size_t lists_cap = 0;
  int32_t* h_counter = nullptr;
  double* h_total = nullptr;
  hipEvent_t mask_copied = nullptr;
  hipStream_t own_stream = nullptr;
};

// A context owns the condition word and caches the device blocks and host kits of freed
// plans, so that building a plan again (a serving loop rebuilds its merged plan whenever
// the resident set changes) neither allocates nor frees device memory -- hipFree would
// synchronise the device every time.  It lives until its handle and every plan made from
// it are released.
struct cel_ctx {
  int device;
  cel_options opt;
  int32_t* d_err = nullptr;       // device condition word (CEL_DEVERR_*), shared by the plans
  double* d_ctable = nullptr;     // data constants of small counts (k_pixconst)
  int refs = 1;                   // the caller's handle + one per live plan
  std::multimap<size_t, void*> cache;   // free device blocks by size
  size_t cache_bytes = 0;
  std::vector<HostKit> kits;
  char* h_stage = nullptr;        // pinned staging buffer for plan uploads
  size_t stage_cap = 0;
};

struct cel_plan {
  int device = 0;
  cel_options opt;
  int S = 0, N = 0, P = 0;
  int64_t n_units = 0, n_tasks = 0;
  // sizes the per-call scratch is allocated for (>= S, P, n_tasks, n_units; grown by
  // cel_plan_append), and the element capacity of each persistent device array that an
  // append may grow, by the address of its pointer field (absent: exactly its count)
  int64_t cap_S = 0, cap_P = 0, cap_T = 0, cap_U = 0;
  std::map<const void*, size_t> dev_cap;
  void* pack_base = nullptr;        // the one block holding the plan's small tables and lists
  std::vector<size_t> cls_cap[3];   // capacities of the per-colour source, patch, item lists
  int nexp = 0, ndev = 0;
  // host copies
  std::vector<cel_image> images_h;
  std::vector<celmi::DPatch> patches_h;
  std::vector<int32_t> patch_ptr_h, nbr_idx_h, order_h;
  std::vector<celmi::DMapTask> map_tasks_h;   // moment-map work items, in launch order
  std::vector<celmi::DTask> tasks_h;
  std::vector<std::vector<int>> adj;
  std::vector<int> colour;
  int n_colours = 0;
  // per colour class c < n_colours: its sources, patches and work items (cost order); entry
  // n_colours (Newton scratch) holds the sources stepped by one cel_newton_step call
  std::vector<std::vector<int32_t>> class_patches, class_tasks, class_src;
  celmi::DPrior prior_h;
  celmi::DProfiles prof_h;
  // device tables
  celmi::DPatch* d_patches = nullptr;
  cel_image* d_images = nullptr;
  int32_t* d_nbr = nullptr;
  celmi::DTask* d_tasks = nullptr;
  int32_t* d_order = nullptr;
  celmi::DMapTask* d_map_tasks = nullptr;
  int32_t* d_patch_ptr = nullptr;
  int32_t* d_npsf = nullptr;
  celmi::DPrior* d_prior = nullptr;
  celmi::DProfiles* d_prof = nullptr;
  float2* d_xs = nullptr;
  double2* d_xs64 = nullptr;    // only with float64 pixel / Hessian options
  float2* d_maps = nullptr;     // (E_s, V_s) of each patch's source at the base parameters
  double2* d_maps64 = nullptr;
  double* d_pixconst = nullptr;
  double* d_skymin = nullptr;     // per patch: smallest sky value
  double* d_patch_psf = nullptr;  // per patch PSF mixtures [P][kMaxPsf][6] (null: the image's)
  int32_t* d_err = nullptr;       // the context's condition word
  double* d_total = nullptr;
  std::vector<int32_t*> d_class_patches, d_class_tasks, d_class_src;
  // per-variant scratch
  int nv_f = 0, nv_d = 0, nv_slots = 0;
  celmi::Table<float>* tables_f = nullptr;
  celmi::Table<double>* tables_d = nullptr;
  double* slots = nullptr;
  double* v_local = nullptr;
  double* v_own = nullptr;
  double* v_grad = nullptr;
  // Newton scratch
  bool newton_ready = false;
  double* d_theta_trial = nullptr;
  double* d_pred = nullptr;
  double* d_step_norm = nullptr;
  double* d_npix = nullptr;
  int32_t* d_colour = nullptr;
  uint8_t* d_trial_active = nullptr;
  uint8_t* d_mask = nullptr;
  int32_t* d_counter = nullptr;
  uint8_t* h_mask = nullptr;      // pinned
  int32_t* h_lists = nullptr;     // pinned, S + P + n_tasks entries
  size_t lists_cap = 0;
  int32_t* h_counter = nullptr;   // pinned
  double* h_total = nullptr;      // pinned
  hipEvent_t mask_copied = nullptr;
  hipStream_t own_stream = nullptr;
  struct Graph {
    hipGraphExec_t exec = nullptr;
    double* theta = nullptr;
    double* radius = nullptr;
    int32_t* status = nullptr;
    hipStream_t stream = nullptr;
  };
  std::vector<Graph> graphs;
  bool marking = false;
  // variant bookkeeping: central-difference variants on/off, index of the trial variant
  int fd_mode = 1;
  int trial_variant = celmi::kVariants - 1;
  double* d_hslots = nullptr;     // analytic Hessian partial sums [n_tasks][80]
  int32_t* d_step_src = nullptr;      // a Newton step's sources, patches and work items
  int32_t* d_step_patches = nullptr;
  int32_t* d_step_tasks = nullptr;
  double* d_hess = nullptr;       // per-source pixel Hessians [S][27][27]
  double* d_hpart = nullptr;      // per-source partial Hessian sums [S][kHessParts][kHessPartN]
  // point-likelihood scratch: parameters of the fixed point and of pt_cap candidates
  // [(pt_cap + 1)][S][32], candidate support flags [pt_cap][S]
  double* d_pt_theta = nullptr;
  uint8_t* d_pt_ok = nullptr;
  int pt_cap = 0;
  // MCMC source step scratch (grow-only): chain records (bytes), candidate rows, their log
  // likelihoods and log priors, selection + mask + counter words, samples, temperatures
  char* mc_chains = nullptr;
  double* mc_cand = nullptr;
  double* mc_vals = nullptr;
  uint8_t* mc_act = nullptr;       // per (candidate, source): the chain still runs
  int32_t* mc_sel = nullptr;
  double* mc_samples = nullptr;
  double* mc_gamma = nullptr;
  size_t mc_chains_cap = 0, mc_cand_cap = 0, mc_vals_cap = 0, mc_sel_cap = 0, mc_samples_cap = 0, mc_gamma_cap = 0, mc_act_cap = 0;
  struct Block {
    void* ptr;
    size_t bytes;
  };
  std::vector<Block> allocs;
  cel_ctx* ctx = nullptr;
  size_t mask_cap = 0;
  // measurement: events per recorded evaluation (start, tables, maps, pixels, end)
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::array<hipEvent_t, 5>> ev_rec;
};

namespace celmi {
// the Hessian's patch sums are split over kHessParts wavefronts per source, each writing
// a record of kHessPartN doubles (27 x 27 Hessian, 27 gradient entries, the local sum)
constexpr int kHessParts = 4;
constexpr int kHessPartN = 27 * 27 + 27 + 1 + 3;
cel_options default_options();
void plan_release(cel_plan* p);
void ctx_release(cel_ctx* c);
// a device block of at least `bytes` from the context's cache, else newly allocated
cel_status ctx_alloc(cel_ctx* c, size_t bytes, void** ptr, size_t* got);
cel_status ensure_variants(cel_plan* p, int nv, bool fp64);
// a device block of `bytes` owned by the plan (freed with it)
cel_status plan_alloc(cel_plan* p, size_t bytes, void** ptr);
// give a block the plan owns back to the context (no work may still use it)
void plan_untrack(cel_plan* p, void* ptr);
// (local_out / grad_out: where variant 0's local objectives and gradients go when nv == 1;
// null = the plan's per-variant arrays)
hipError_t eval_any(cel_plan* p, const double* theta, const double* theta_trial, int v0, int nv, bool grad, int cls,
                    const uint8_t* active, hipStream_t sm, bool prep_base, bool fp64, double* local_out = nullptr,
                    double* grad_out = nullptr);
hipError_t plain_eval(cel_plan* p, const double* theta, hipStream_t sm, bool fp64);
// component tables at the iterate for every patch and the neighbour moment maps (hess: with
// the exact Hessian's records)
hipError_t prep_base(cel_plan* p, const double* theta, hipStream_t sm, bool fp64, bool hess = false);
// component tables at the iterate for the patches of colour class cls only (sources flagged
// in active); the maps are left as they are
hipError_t prep_class(cel_plan* p, const double* theta, int cls, const uint8_t* active, hipStream_t sm, bool fp64,
                      bool hess = false);
// record a phase boundary event (k = 0..4) of the current evaluation when timing is on
void phase_mark(cel_plan* p, int k, hipStream_t sm);
cel_status ensure_newton(cel_plan* p);
// the work items at p->opt.chunk_pixels (host tables: items, patch ranges, launch order,
// moment-map items, per-colour item lists)
cel_status build_tiling(cel_plan* p);
// re-cut a prepared plan's work items at `chunk` pixels: host tables, their device copies and
// the per-call scratch sized by the item count (waits for the device first)
cel_status plan_retile(cel_plan* p, int chunk, hipStream_t sm);
// Stage a selection of sources (m[s] != 0) for a batched call: the mask to p->d_mask and,
// when as_class, the union of the selected sources as the step class (index n_colours) --
// its source, patch and work-item lists -- through the plan's pinned buffers.  Waits for the
// previous call's copies out of those buffers and records p->mask_copied after its own.
hipError_t stage_selection(cel_plan* p, const std::vector<uint8_t>& m, bool as_class, hipStream_t sm);
// global ELBO at theta into p->d_total (tables, ELBO-only pixel pass, finalisation, total)
hipError_t launch_total_after_eval(cel_plan* p, const double* theta, hipStream_t sm);
// Point likelihood passes: point_setup stages the selection (m[s] != 0) and the neighbour
// maps at z_fixed, with scratch for `chunk` candidates per launch (<= kVariants); then each
// point_loglik writes ll[c][s] for the selected sources of n_cand candidate rows z_cand
// (act: optional [n_cand][S] flags; a (candidate, source) flagged 0 is not evaluated and its
// ll entry is left as it was; mark_support: set -infinity for candidates outside the
// support, which a caller that also takes the prior density, -infinity there, may skip).
cel_status point_setup(cel_plan* p, const double* z_fixed, const std::vector<uint8_t>& m, int chunk, hipStream_t sm);
hipError_t point_loglik(cel_plan* p, int n_cand, const double* z_cand, double* ll, hipStream_t sm,
                        const uint8_t* act = nullptr, bool mark_support = true);
}  // namespace celmi
