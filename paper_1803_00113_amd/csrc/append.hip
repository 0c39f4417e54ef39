// cel_plan_append: add a problem's sources, images and patches to an existing plan at a cost
// that depends on the added part only (amortised), not on what the plan already holds.
//
// The part is prepared on its own (validation, overlap lists, colouring, work items, pixel
// staging and data constants: cel_prepare), then spliced into the plan: its host tables
// are appended with their ids shifted; every persistent device array grows by doubling
// (old contents copied on the device) and receives the part's slice.  The part's patches
// lie in its own images, so no source of the part overlaps one already in the plan: the
// overlap graph gains no edge across the two, and the greedy colouring of the whole
// (ascending id) restricted to the part equals the part's own.  Per-call scratch (component
// tables, moment maps, slot rows, Newton and likelihood buffers) is sized by the plan's
// capacities, which double when an append exceeds them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device.h"
#include "plan.h"

using namespace celmi;

namespace {

struct Growth {
  cel_plan* p;
  hipStream_t sm;
  std::vector<void*> old_blocks;   // returned to the context once the copies are done

  // ensure *field holds new_n elements, its first old_n kept
  template <typename X>
  cel_status grow(X** field, size_t old_n, size_t new_n, size_t* cap_slot = nullptr) {
    size_t cap = old_n;
    if (cap_slot) {
      cap = std::max(*cap_slot, old_n);
    } else {
      auto it = p->dev_cap.find(field);
      if (it != p->dev_cap.end()) cap = it->second;
    }
    if (new_n <= cap && *field) return CEL_OK;
    const size_t ncap = std::max<size_t>({new_n, 2 * cap, 16});
    void* q = nullptr;
    cel_status st = plan_alloc(p, ncap * sizeof(X), &q);
    if (st) return st;
    if (old_n && *field &&
        hipMemcpyAsync(q, *field, old_n * sizeof(X), hipMemcpyDeviceToDevice, sm) != hipSuccess)
      return CEL_EHIP;
    // a block of its own goes back to the context; an array inside the plan's packed
    // block stays there (plan_untrack never releases that block)
    if (*field) old_blocks.push_back(*field);
    *field = static_cast<X*>(q);
    if (cap_slot)
      *cap_slot = ncap;
    else
      p->dev_cap[field] = ncap;
    return CEL_OK;
  }

  template <typename X>
  cel_status put(X* dst, const X* src, size_t n, hipMemcpyKind kind) {
    if (!n) return CEL_OK;
    return hipMemcpyAsync(dst, src, n * sizeof(X), kind, sm) == hipSuccess ? CEL_OK : CEL_EHIP;
  }
};

// Give up the per-call scratch sized by the plan's capacities (component tables, slot rows,
// per-source outputs, moment maps, point and Newton buffers); the caller allocates it again
// at the new capacities.  The blocks go back once the queued copies are done.
cel_status drop_scratch(Growth& g) {
  cel_plan* p = g.p;
  for (void* b : {(void*)p->tables_f, (void*)p->tables_d, (void*)p->slots, (void*)p->v_local, (void*)p->v_own,
                  (void*)p->v_grad, (void*)p->d_maps, (void*)p->d_maps64, (void*)p->d_pt_theta, (void*)p->d_pt_ok})
    g.old_blocks.push_back(b);
  p->tables_f = nullptr;
  p->tables_d = nullptr;
  p->slots = p->v_local = p->v_own = p->v_grad = nullptr;
  p->nv_f = p->nv_d = p->nv_slots = 0;
  p->d_pt_theta = nullptr;
  p->d_pt_ok = nullptr;
  p->pt_cap = 0;
  if (p->newton_ready) {
    for (void* b : {(void*)p->d_theta_trial, (void*)p->d_pred, (void*)p->d_step_norm, (void*)p->d_trial_active,
                    (void*)p->d_mask, (void*)p->d_counter, (void*)p->d_hslots, (void*)p->d_step_src,
                    (void*)p->d_step_patches, (void*)p->d_step_tasks, (void*)p->d_hess, (void*)p->d_hpart})
      g.old_blocks.push_back(b);
    p->newton_ready = false;
  }
  const bool m64 = p->d_maps64 != nullptr;
  p->d_maps = nullptr;
  p->d_maps64 = nullptr;
  void* b = nullptr;
  cel_status st = plan_alloc(p, (size_t)std::max<int64_t>(p->cap_U, 1) * sizeof(float2), &b);
  if (st) return st;
  p->d_maps = static_cast<float2*>(b);
  if (m64) {
    if ((st = plan_alloc(p, (size_t)std::max<int64_t>(p->cap_U, 1) * sizeof(double2), &b))) return st;
    p->d_maps64 = static_cast<double2*>(b);
  }
  return CEL_OK;
}

// After a change of the class lists or of the capacities: the evaluation scratch exists
// again, the Newton scratch too when the plan had it, and the step class (entry n_colours of
// the class lists) points at the Newton step's lists.  Captured sweep graphs, which hold the
// old arrays and class sizes, are dropped.
cel_status restore_scratch(cel_plan* p, bool had_step) {
  cel_status st = ensure_variants(p, 1, p->opt.pixel_fp64 != 0);
  if (st) return st;
  if (had_step) {
    if (p->newton_ready) {
      p->class_src.resize(p->n_colours + 1);
      p->class_patches.resize(p->n_colours + 1);
      p->class_tasks.resize(p->n_colours + 1);
      p->d_class_src.resize(p->n_colours + 1);
      p->d_class_patches.resize(p->n_colours + 1);
      p->d_class_tasks.resize(p->n_colours + 1);
      p->d_class_src[p->n_colours] = p->d_step_src;
      p->d_class_patches[p->n_colours] = p->d_step_patches;
      p->d_class_tasks[p->n_colours] = p->d_step_tasks;
    } else if ((st = ensure_newton(p))) {
      return st;
    }
  }
  for (auto& gr : p->graphs)
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
  p->graphs.clear();
  return CEL_OK;
}

}  // namespace

extern "C" void cel_plan_free(cel_plan* plan);

extern "C" cel_status cel_plan_append(cel_ctx* ctx, cel_plan* p, const cel_problem* part, void* stream) {
  if (!ctx || !p || !part || p->ctx != ctx) return CEL_EINVAL;
  if (p->d_patch_psf || part->patch_psf) return CEL_EUNSUPPORTED;
  if ((int64_t)p->N + part->n_images >= (1 << 20) || (int64_t)p->P + part->n_patches >= (1 << 24) ||
      (int64_t)p->S + part->n_sources >= (1 << 30))
    return CEL_EUNSUPPORTED;
  hipStream_t sm = (hipStream_t)stream;
  cel_plan* q = nullptr;
  cel_status st = cel_prepare(ctx, part, &q, stream);
  if (st) return st;
  if (std::memcmp(&q->prior_h, &p->prior_h, sizeof(DPrior)) || std::memcmp(&q->prof_h, &p->prof_h, sizeof(DProfiles)) ||
      p->n_tasks + q->n_tasks > ((int64_t)1 << 30)) {
    const bool big = p->n_tasks + q->n_tasks > ((int64_t)1 << 30);
    cel_plan_free(q);
    return big ? CEL_EUNSUPPORTED : CEL_EINVAL;
  }
  if (hipSetDevice(p->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    cel_plan_free(q);
    return CEL_EHIP;
  }
  // the part's work items are cut at the plan's size (cel_tune may have changed it)
  if ((st = plan_retile(q, p->opt.chunk_pixels, sm))) {
    cel_plan_free(q);
    return st;
  }
  const int S0 = p->S, N0 = p->N, P0 = p->P;
  const int64_t U0 = p->n_units, T0 = p->n_tasks;
  const int E0 = (int)p->nbr_idx_h.size(), M0 = (int)p->map_tasks_h.size();
  // --- host tables --------------------------------------------------------------------
  p->images_h.insert(p->images_h.end(), q->images_h.begin(), q->images_h.end());
  for (DPatch d : q->patches_h) {
    d.src += S0;
    d.img += N0;
    d.off += U0;
    d.nbr_begin += E0;
    d.nbr_end += E0;
    d.task_begin += (int)T0;
    d.task_end += (int)T0;
    p->patches_h.push_back(d);
  }
  for (int v : q->nbr_idx_h) p->nbr_idx_h.push_back(v + P0);
  for (DTask t : q->tasks_h) {
    t.patch += P0;
    p->tasks_h.push_back(t);
  }
  for (int v : q->order_h) p->order_h.push_back(v + (int)T0);
  for (DMapTask m : q->map_tasks_h) {
    m.patch += P0;
    p->map_tasks_h.push_back(m);
  }
  for (int s = 1; s <= q->S; ++s) p->patch_ptr_h.push_back(q->patch_ptr_h[s] + P0);
  for (const auto& a : q->adj) {
    std::vector<int> b(a);
    for (int& t : b) t += S0;
    p->adj.push_back(b);
  }
  for (int c : q->colour) p->colour.push_back(c);
  // the per-colour lists (the step class, entry n_colours, is set again below)
  const bool had_step = p->newton_ready;
  const int C0 = p->n_colours, C1 = std::max(C0, q->n_colours);
  p->class_src.resize(C0);
  p->class_patches.resize(C0);
  p->class_tasks.resize(C0);
  p->d_class_src.resize(C0);
  p->d_class_patches.resize(C0);
  p->d_class_tasks.resize(C0);
  for (int k = 0; k < 3; ++k) p->cls_cap[k].resize(C0, 0);
  std::vector<size_t> cls_old[3];
  for (int c = 0; c < C0; ++c) {
    cls_old[0].push_back(p->class_src[c].size());
    cls_old[1].push_back(p->class_patches[c].size());
    cls_old[2].push_back(p->class_tasks[c].size());
  }
  p->class_src.resize(C1);
  p->class_patches.resize(C1);
  p->class_tasks.resize(C1);
  p->d_class_src.resize(C1, nullptr);
  p->d_class_patches.resize(C1, nullptr);
  p->d_class_tasks.resize(C1, nullptr);
  for (int k = 0; k < 3; ++k) {
    p->cls_cap[k].resize(C1, 0);
    cls_old[k].resize(C1, 0);
  }
  for (int c = 0; c < q->n_colours; ++c) {
    for (int v : q->class_src[c]) p->class_src[c].push_back(v + S0);
    for (int v : q->class_patches[c]) p->class_patches[c].push_back(v + P0);
    for (int v : q->class_tasks[c]) p->class_tasks[c].push_back(v + (int)T0);
  }
  p->S += q->S;
  p->N += q->N;
  p->P += q->P;
  p->n_units += q->n_units;
  p->n_tasks += q->n_tasks;
  p->n_colours = C1;
  const int S = p->S, N = p->N, P = p->P;
  const int64_t U = p->n_units, T = p->n_tasks;
  // --- persistent device arrays ---------------------------------------------------------
  Growth g{p, sm, {}};
  std::vector<int32_t> npsf(q->N), col(q->S);
  std::vector<double> npix(q->S, 0.0);
  for (int n = 0; n < q->N; ++n) npsf[n] = q->images_h[n].n_psf;
  for (int s = 0; s < q->S; ++s) col[s] = q->colour[s];
  for (const DPatch& d : q->patches_h) npix[d.src] += (double)d.w * d.h;
  const bool xs64 = p->d_xs64 != nullptr;
  const auto H2D = hipMemcpyHostToDevice, D2D = hipMemcpyDeviceToDevice;
  if ((st = g.grow(&p->d_patches, P0, P)) || (st = g.put(p->d_patches + P0, p->patches_h.data() + P0, P - P0, H2D)) ||
      (st = g.grow(&p->d_images, N0, N)) || (st = g.put(p->d_images + N0, p->images_h.data() + N0, N - N0, H2D)) ||
      (st = g.grow(&p->d_nbr, E0, p->nbr_idx_h.size())) ||
      (st = g.put(p->d_nbr + E0, p->nbr_idx_h.data() + E0, p->nbr_idx_h.size() - E0, H2D)) ||
      (st = g.grow(&p->d_tasks, T0, T)) || (st = g.put(p->d_tasks + T0, p->tasks_h.data() + T0, T - T0, H2D)) ||
      (st = g.grow(&p->d_order, T0, T)) || (st = g.put(p->d_order + T0, p->order_h.data() + T0, T - T0, H2D)) ||
      (st = g.grow(&p->d_map_tasks, M0, p->map_tasks_h.size())) ||
      (st = g.put(p->d_map_tasks + M0, p->map_tasks_h.data() + M0, p->map_tasks_h.size() - M0, H2D)) ||
      (st = g.grow(&p->d_patch_ptr, S0 + 1, S + 1)) ||
      (st = g.put(p->d_patch_ptr + S0 + 1, p->patch_ptr_h.data() + S0 + 1, S - S0, H2D)) ||
      (st = g.grow(&p->d_npsf, N0, N)) || (st = g.put(p->d_npsf + N0, npsf.data(), npsf.size(), H2D)) ||
      (st = g.grow(&p->d_npix, S0, S)) || (st = g.put(p->d_npix + S0, npix.data(), npix.size(), H2D)) ||
      (st = g.grow(&p->d_colour, S0, S)) || (st = g.put(p->d_colour + S0, col.data(), col.size(), H2D)) ||
      (st = g.grow(&p->d_xs, U0, U)) || (st = g.put(p->d_xs + U0, q->d_xs, U - U0, D2D)) ||
      (xs64 && ((st = g.grow(&p->d_xs64, U0, U)) || (st = g.put(p->d_xs64 + U0, q->d_xs64, U - U0, D2D)))) ||
      (st = g.grow(&p->d_pixconst, 2 * (size_t)P0, 2 * (size_t)P)) ||
      (st = g.put(p->d_pixconst + 2 * P0, q->d_pixconst, 2 * (size_t)(P - P0), D2D)) ||
      (st = g.grow(&p->d_skymin, P0, P)) || (st = g.put(p->d_skymin + P0, q->d_skymin, P - P0, D2D))) {
    cel_plan_free(q);
    return st;
  }
  for (int c = 0; c < C1 && !st; ++c) {
    const size_t ns = p->class_src[c].size(), np = p->class_patches[c].size(), nt = p->class_tasks[c].size();
    if ((st = g.grow(&p->d_class_src[c], cls_old[0][c], ns, &p->cls_cap[0][c])) ||
        (st = g.put(p->d_class_src[c] + cls_old[0][c], p->class_src[c].data() + cls_old[0][c], ns - cls_old[0][c], H2D)) ||
        (st = g.grow(&p->d_class_patches[c], cls_old[1][c], np, &p->cls_cap[1][c])) ||
        (st = g.put(p->d_class_patches[c] + cls_old[1][c], p->class_patches[c].data() + cls_old[1][c],
                    np - cls_old[1][c], H2D)) ||
        (st = g.grow(&p->d_class_tasks[c], cls_old[2][c], nt, &p->cls_cap[2][c])) ||
        (st = g.put(p->d_class_tasks[c] + cls_old[2][c], p->class_tasks[c].data() + cls_old[2][c], nt - cls_old[2][c],
                    H2D)))
      break;
  }
  if (st) {
    cel_plan_free(q);
    return st;
  }
  // --- per-call scratch: regrown when the plan outgrows its capacities -------------------
  if (S > p->cap_S || P > p->cap_P || T > p->cap_T || U > p->cap_U) {
    p->cap_S = std::max<int64_t>(S, 2 * p->cap_S);
    p->cap_P = std::max<int64_t>(P, 2 * p->cap_P);
    p->cap_T = std::max<int64_t>(T, 2 * p->cap_T);
    p->cap_U = std::max<int64_t>(U, 2 * p->cap_U);
    if ((st = drop_scratch(g))) {
      cel_plan_free(q);
      return st;
    }
  }
  // the evaluation calls allocate nothing: their scratch exists before they are made
  if ((st = restore_scratch(p, had_step))) {
    cel_plan_free(q);
    return st;
  }
  hipError_t e = hipStreamSynchronize(sm);
  for (void* b : g.old_blocks) plan_untrack(p, b);
  cel_plan_free(q);
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

cel_status celmi::plan_retile(cel_plan* p, int chunk, hipStream_t sm) {
  if (chunk == p->opt.chunk_pixels) return CEL_OK;
  if (hipSetDevice(p->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return CEL_EHIP;
  const int keep = p->opt.chunk_pixels;
  const bool had_step = p->newton_ready;
  p->opt.chunk_pixels = chunk;
  cel_status st = build_tiling(p);
  if (st) {   // too many items: the old cut stays
    p->opt.chunk_pixels = keep;
    (void)build_tiling(p);
    return st;
  }
  const int64_t T = p->n_tasks;
  const int C = p->n_colours;
  Growth g{p, sm, {}};
  const auto H2D = hipMemcpyHostToDevice;
  // the patches' item ranges changed in place; the item lists are written whole
  if ((st = g.put(p->d_patches, p->patches_h.data(), p->patches_h.size(), H2D)) ||
      (st = g.grow(&p->d_tasks, 0, T)) || (st = g.put(p->d_tasks, p->tasks_h.data(), T, H2D)) ||
      (st = g.grow(&p->d_order, 0, T)) || (st = g.put(p->d_order, p->order_h.data(), T, H2D)) ||
      (st = g.grow(&p->d_map_tasks, 0, p->map_tasks_h.size())) ||
      (st = g.put(p->d_map_tasks, p->map_tasks_h.data(), p->map_tasks_h.size(), H2D)))
    return st;
  for (int k = 0; k < 3; ++k) p->cls_cap[k].resize(std::max<size_t>(p->cls_cap[k].size(), C), 0);
  for (int c = 0; c < C; ++c) {
    const size_t nt = p->class_tasks[c].size();
    if ((st = g.grow(&p->d_class_tasks[c], 0, nt, &p->cls_cap[2][c])) ||
        (st = g.put(p->d_class_tasks[c], p->class_tasks[c].data(), nt, H2D)))
      return st;
  }
  if (T > p->cap_T) {
    p->cap_T = T;
    if ((st = drop_scratch(g))) return st;
  }
  if ((st = restore_scratch(p, had_step))) return st;
  hipError_t e = hipStreamSynchronize(sm);
  for (void* b : g.old_blocks) plan_untrack(p, b);
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}
