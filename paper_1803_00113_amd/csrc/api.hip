// Host side of the celmi C ABI: validation, plan building and launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "plan.h"

using namespace celmi;

extern "C" const char* cel_strerror(cel_status s) {
  switch (s) {
    case CEL_OK: return "ok";
    case CEL_EINVAL: return "invalid argument";
    case CEL_ENOMEM: return "device allocation failed";
    case CEL_EHIP: return "HIP runtime error";
    case CEL_EUNSUPPORTED: return "unsupported size or option";
    case CEL_ESCRATCH: return "the call needs more scratch than the static buffer holds (CEL_STATIC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

namespace celmi {

cel_options default_options() {
  cel_options o;
  std::memset(&o, 0, sizeof(o));
  o.pixels_per_lane = 2;
  o.chunk_pixels = 512;
  o.map_pixels_per_lane = 4;
  o.fd_step = 0.0;   // resolved in merge_options: 1e-2 (float32 pixels), 1e-3 (float64)
  o.radius0 = 1.0;
  o.radius_max = 100.0;
  o.eta = 0.1;
  o.gtol = 1e-6;
  o.ftol = 1e-9;
  o.radius_min = 1e-8;
  return o;
}

static cel_options merge_options(const cel_options* in) {
  cel_options o = default_options();
  if (!in) return o;
  if (in->pixels_per_lane) o.pixels_per_lane = in->pixels_per_lane;
  if (in->chunk_pixels) o.chunk_pixels = in->chunk_pixels;
  if (in->map_pixels_per_lane != 0) o.map_pixels_per_lane = in->map_pixels_per_lane;
  o.pixel_fp64 = in->pixel_fp64;
  o.hessian_fp64 = in->hessian_fp64;
  o.hessian_fd = in->hessian_fd;
  if (in->fd_step > 0) o.fd_step = in->fd_step;
  if (in->radius0 > 0) o.radius0 = in->radius0;
  if (in->radius_max > 0) o.radius_max = in->radius_max;
  if (in->eta > 0) o.eta = in->eta;
  if (in->gtol > 0) o.gtol = in->gtol;
  if (in->ftol > 0) o.ftol = in->ftol;
  if (in->radius_min > 0) o.radius_min = in->radius_min;
  o.timing = in->timing;
  return o;
}

static void resolve_fd_step(cel_options& o) {
  // central differences of a gradient carrying float32 rounding noise eps: error ~ eps/h +
  // h^2 |f'''|, so float32 gradients take a larger step than float64 ones
  if (!(o.fd_step > 0)) o.fd_step = (o.pixel_fp64 || o.hessian_fp64) ? 1e-3 : 1e-2;
}

static bool finite(double x) { return std::isfinite(x); }

// inverse and log-determinant of a symmetric positive definite 4x4 matrix (Cholesky)
static bool spd_inverse4(const double in[4][4], double out[4][4], double* logdet) {
  double L[4][4] = {};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = in[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0)) return false;
        L[i][i] = std::sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  *logdet = 0;
  for (int i = 0; i < 4; ++i) *logdet += 2.0 * std::log(L[i][i]);
  // inverse via solving L L^T X = I column by column
  for (int c = 0; c < 4; ++c) {
    double y[4], x[4];
    for (int i = 0; i < 4; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
      y[i] = s / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < 4; ++k) s -= L[k][i] * x[k];
      x[i] = s / L[i][i];
    }
    for (int i = 0; i < 4; ++i) out[i][c] = x[i];
  }
  return true;
}

static cel_status validate(const cel_problem* pr) {
  if (!pr || pr->n_sources < 0 || pr->n_images < 0 || pr->n_patches < 0 || pr->n_pixels < 0 ||
      pr->n_sky_knots < 0)
    return CEL_EINVAL;
  if (pr->n_images > 0 && !pr->images) return CEL_EINVAL;
  if (pr->n_patches > 0 && (!pr->patches || !pr->pixels)) return CEL_EINVAL;
  if (!pr->prior || !pr->profiles) return CEL_EINVAL;
  if (pr->n_sky_knots > 0 && !pr->sky_knots) return CEL_EINVAL;
  // (the neighbour sweep packs image, column and patch id into one 64-bit key)
  if (pr->n_images >= (1 << 20) || pr->n_patches >= (1 << 24)) return CEL_EUNSUPPORTED;
  for (int n = 0; n < pr->n_images; ++n) {
    const cel_image& im = pr->images[n];
    if (im.band < 0 || im.band > 4 || im.H < 1 || im.W < 1 || im.n_psf < 1) return CEL_EINVAL;
    if (im.n_psf > kMaxPsf || im.W > (1 << 20)) return CEL_EUNSUPPORTED;
    for (int k = 0; k < im.n_psf; ++k) {
      const double* q = im.psf[k];
      for (int i = 0; i < 6; ++i)
        if (!finite(q[i])) return CEL_EINVAL;
      if (q[0] < 0 || !(q[3] > 0) || !(q[3] * q[5] - q[4] * q[4] > 0)) return CEL_EINVAL;
    }
    const double det = im.A[0][0] * im.A[1][1] - im.A[0][1] * im.A[1][0];
    if (!finite(det) || det == 0.0 || !finite(im.b[0]) || !finite(im.b[1])) return CEL_EINVAL;
    if (!(im.iota > 0) || !finite(im.iota)) return CEL_EINVAL;
    if (im.sky_qh < 1 || im.sky_qw < 1 || im.sky_off < 0 ||
        im.sky_off + (int64_t)im.sky_qh * im.sky_qw > pr->n_sky_knots)
      return CEL_EINVAL;
    if ((im.sky_qh > 1 && im.H < 2) || (im.sky_qw > 1 && im.W < 2)) return CEL_EINVAL;
    for (int64_t i = 0; i < (int64_t)im.sky_qh * im.sky_qw; ++i) {
      const double v = pr->sky_knots[im.sky_off + i];
      if (!(v > 0) || !finite(v)) return CEL_EINVAL;
    }
  }
  for (int p = 0; p < pr->n_patches; ++p) {
    const cel_patch& q = pr->patches[p];
    if (q.src < 0 || q.src >= pr->n_sources || q.img < 0 || q.img >= pr->n_images) return CEL_EINVAL;
    if (pr->patch_psf) {   // the patch's own PSF mixture: as an image's
      for (int k = 0; k < pr->images[q.img].n_psf; ++k) {
        const double* c = pr->patch_psf + ((int64_t)p * kMaxPsf + k) * 6;
        for (int i = 0; i < 6; ++i)
          if (!finite(c[i])) return CEL_EINVAL;
        if (c[0] < 0 || !(c[3] > 0) || !(c[3] * c[5] - c[4] * c[4] > 0)) return CEL_EINVAL;
      }
    }
    if (q.w < 1 || q.h < 1) return CEL_EINVAL;
    if ((int64_t)q.w * q.h > (int64_t(1) << 22)) return CEL_EUNSUPPORTED;
    const cel_image& im = pr->images[q.img];
    if (q.x0 < 0 || q.y0 < 0 || (int64_t)q.x0 + q.w > im.W || (int64_t)q.y0 + q.h > im.H) return CEL_EINVAL;
    if (q.pix_off < 0 || q.pix_off + (int64_t)q.w * q.h > pr->n_pixels) return CEL_EINVAL;
    if (p > 0) {
      const cel_patch& r = pr->patches[p - 1];
      if (r.src > q.src || (r.src == q.src && r.img >= q.img)) return CEL_EINVAL;
    }
  }
  const cel_prior& pp = *pr->prior;
  if (!(pp.star_prob > 0 && pp.star_prob < 1)) return CEL_EINVAL;
  for (int i = 0; i < 2; ++i) {
    if (!finite(pp.r[i][0]) || !(pp.r[i][1] > 0)) return CEL_EINVAL;
    double sw = 0;
    for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) {
      if (!(pp.c_w[i][j] >= 0)) return CEL_EINVAL;
      sw += pp.c_w[i][j];
      double inv[4][4], ld;
      if (pp.c_w[i][j] > 0 && !spd_inverse4(pp.c_cov[i][j], inv, &ld)) return CEL_EINVAL;
    }
    if (!(std::fabs(sw - 1.0) < 1e-6)) return CEL_EINVAL;
  }
  if (!finite(pp.radius[0]) || !(pp.radius[1] > 0)) return CEL_EINVAL;
  if (!(pp.profile[0] > 0 && pp.profile[1] > 0 && pp.axis[0] > 0 && pp.axis[1] > 0)) return CEL_EINVAL;
  const cel_profiles& pf = *pr->profiles;
  if (pf.n_exp < 1 || pf.n_dev < 1) return CEL_EINVAL;
  if (pf.n_exp > kMaxProf || pf.n_dev > kMaxProf) return CEL_EUNSUPPORTED;
  for (int j = 0; j < pf.n_exp; ++j)
    if (!(pf.exp_alpha[j] >= 0) || !(pf.exp_tau[j] > 0)) return CEL_EINVAL;
  for (int j = 0; j < pf.n_dev; ++j)
    if (!(pf.dev_alpha[j] >= 0) || !(pf.dev_tau[j] > 0)) return CEL_EINVAL;
  return CEL_OK;
}

constexpr size_t kCacheCap = (size_t)8 << 30;   // device bytes a context keeps for reuse

cel_status ctx_alloc(cel_ctx* c, size_t bytes, void** ptr, size_t* got) {
  bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  *ptr = nullptr;
  if (c) {
    auto it = c->cache.lower_bound(bytes);
    if (it != c->cache.end() && it->first <= bytes + bytes / 4 + 65536) {
      *ptr = it->second;
      *got = it->first;
      c->cache_bytes -= it->first;
      c->cache.erase(it);
      return CEL_OK;
    }
  }
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    *ptr = nullptr;
    // drop the cache and try once more
    if (c && !c->cache.empty()) {
      (void)hipDeviceSynchronize();
      for (auto& kv : c->cache) (void)hipFree(kv.second);
      c->cache.clear();
      c->cache_bytes = 0;
      if (hipMalloc(ptr, bytes) == hipSuccess) {
        *got = bytes;
        return CEL_OK;
      }
    }
    *ptr = nullptr;
    return CEL_ENOMEM;
  }
  *got = bytes;
  return CEL_OK;
}

void ctx_release(cel_ctx* c) {
  if (!c || --c->refs > 0) return;
  if (hipSetDevice(c->device) == hipSuccess) {
    (void)hipDeviceSynchronize();
    for (auto& kv : c->cache) (void)hipFree(kv.second);
    for (HostKit& k : c->kits) {
      if (k.mask_copied) (void)hipEventDestroy(k.mask_copied);
      if (k.own_stream) (void)hipStreamDestroy(k.own_stream);
      if (k.h_mask) (void)hipHostFree(k.h_mask);
      if (k.h_lists) (void)hipHostFree(k.h_lists);
      if (k.h_counter) (void)hipHostFree(k.h_counter);
      if (k.h_total) (void)hipHostFree(k.h_total);
    }
    if (c->d_err) (void)hipFree(c->d_err);
    if (c->d_ctable) (void)hipFree(c->d_ctable);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
  }
  delete c;
}

void plan_release(cel_plan* p) {
  if (!p) return;
  // work of this plan may still be in flight on the caller's streams: finish it before
  // its memory is reused (one synchronisation instead of one per freed block)
  if (!p->allocs.empty() || p->mask_copied) (void)hipDeviceSynchronize();
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  cel_ctx* c = p->ctx;
  if (p->mask_copied) {
    HostKit k;
    k.h_mask = p->h_mask;
    k.mask_cap = p->mask_cap;
    k.h_lists = p->h_lists;
    k.lists_cap = p->lists_cap;
    k.h_counter = p->h_counter;
    k.h_total = p->h_total;
    k.mask_copied = p->mask_copied;
    k.own_stream = p->own_stream;
    if (c) {
      c->kits.push_back(k);
    } else {
      (void)hipEventDestroy(k.mask_copied);
      if (k.own_stream) (void)hipStreamDestroy(k.own_stream);
      if (k.h_mask) (void)hipHostFree(k.h_mask);
      if (k.h_lists) (void)hipHostFree(k.h_lists);
      if (k.h_counter) (void)hipHostFree(k.h_counter);
      if (k.h_total) (void)hipHostFree(k.h_total);
    }
  }
  for (auto& b : p->allocs) {
    if (c && c->cache_bytes + b.bytes <= kCacheCap) {
      c->cache.emplace(b.bytes, b.ptr);
      c->cache_bytes += b.bytes;
    } else {
      (void)hipFree(b.ptr);
    }
  }
  for (auto& r : p->ev_rec)
    for (hipEvent_t e : r) p->ev_pool.push_back(e);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
  ctx_release(c);
}

void phase_mark(cel_plan* p, int k, hipStream_t sm) {
  if (!p->opt.timing || !p->marking) return;
  if (k == 0) {
    std::array<hipEvent_t, 5> r;
    for (int i = 0; i < 5; ++i) {
      if (p->ev_pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        p->ev_pool.push_back(e);
      }
      r[i] = p->ev_pool.back();
      p->ev_pool.pop_back();
    }
    p->ev_rec.push_back(r);
  }
  if (p->ev_rec.empty()) return;
  (void)hipEventRecord(p->ev_rec.back()[k], sm);
}

template <typename X>
static cel_status track(cel_plan* p, X** ptr, size_t n) {
  void* q = nullptr;
  size_t got = 0;
  cel_status st = ctx_alloc(p->ctx, std::max<size_t>(n, 1) * sizeof(X), &q, &got);
  *ptr = static_cast<X*>(q);
  if (!st) p->allocs.push_back({q, got});
  return st;
}

cel_status plan_alloc(cel_plan* p, size_t bytes, void** ptr) {
  size_t got = 0;
  cel_status st = ctx_alloc(p->ctx, bytes, ptr, &got);
  if (!st) p->allocs.push_back({*ptr, got});
  return st;
}

void plan_untrack(cel_plan* p, void* ptr) {
  // (the packed block holds many arrays: it lives as long as the plan)
  if (!ptr || ptr == p->pack_base) return;
  for (size_t i = 0; i < p->allocs.size(); ++i) {
    if (p->allocs[i].ptr != ptr) continue;
    const cel_plan::Block b = p->allocs[i];
    p->allocs.erase(p->allocs.begin() + i);
    cel_ctx* c = p->ctx;
    if (c && c->cache_bytes + b.bytes <= kCacheCap) {
      c->cache.emplace(b.bytes, b.ptr);
      c->cache_bytes += b.bytes;
    } else {
      (void)hipFree(b.ptr);
    }
    return;
  }
}

template <typename X>
static cel_status track_upload(cel_plan* p, X** ptr, const std::vector<X>& v) {
  cel_status st = track(p, ptr, v.size());
  if (st) return st;
  if (!v.empty() && hipMemcpy(*ptr, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice) != hipSuccess)
    return CEL_EHIP;
  return CEL_OK;
}

// Host arrays copied to the device in one transfer: each gets its own 256-byte aligned
// slice of one tracked block (one synchronous copy instead of one per array).
struct UploadPack {
  struct Item {
    std::function<void(char*)> set;
    const void* src;
    size_t bytes, off;
  };
  std::vector<Item> items;
  size_t total = 0;
  template <typename X>
  void add(X** dst, const std::vector<X>& v) {
    const size_t off = (total + 255) & ~(size_t)255, bytes = v.size() * sizeof(X);
    items.push_back({[dst](char* q) { *dst = reinterpret_cast<X*>(q); }, v.data(), bytes, off});
    total = off + std::max<size_t>(bytes, 1);
  }
};

static cel_status upload_pack(cel_plan* p, UploadPack& pk, hipStream_t sm) {
  char* base = nullptr;
  cel_status st = track(p, &base, pk.total);
  if (st) return st;
  p->pack_base = base;
  // staged through the context's pinned buffer (grown when a larger plan needs it)
  cel_ctx* c = p->ctx;
  if (c->stage_cap < pk.total) {
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    c->h_stage = nullptr;
    c->stage_cap = 0;
    const size_t cap = std::max<size_t>(pk.total + pk.total / 4, (size_t)1 << 20);
    if (hipHostMalloc((void**)&c->h_stage, cap) != hipSuccess) {
      c->h_stage = nullptr;
      return CEL_ENOMEM;
    }
    c->stage_cap = cap;
  }
  for (auto& it : pk.items) {
    if (it.bytes) std::memcpy(c->h_stage + it.off, it.src, it.bytes);
    it.set(base + it.off);
  }
  if (hipMemcpyAsync(base, c->h_stage, pk.total, hipMemcpyHostToDevice, sm) != hipSuccess ||
      hipStreamSynchronize(sm) != hipSuccess)
    return CEL_EHIP;
  return CEL_OK;
}

// grow the per-variant scratch (tables, slots, per-source outputs) to hold nv variants
cel_status ensure_variants(cel_plan* p, int nv, bool fp64) {
  if (fp64 ? (p->nv_d >= nv) : (p->nv_f >= nv)) {
    if (p->nv_slots >= nv) return CEL_OK;
  }
  cel_status st;
  if (fp64 && p->nv_d < nv) {
    if ((st = track(p, &p->tables_d, (size_t)nv * std::max<int64_t>(p->cap_P, 1)))) return st;
    p->nv_d = nv;
  }
  if (!fp64 && p->nv_f < nv) {
    if ((st = track(p, &p->tables_f, (size_t)nv * std::max<int64_t>(p->cap_P, 1)))) return st;
    p->nv_f = nv;
  }
  if (p->nv_slots < nv) {
    if ((st = track(p, &p->slots, (size_t)nv * std::max<int64_t>(p->cap_T, 1) * kSlots))) return st;
    if ((st = track(p, &p->v_local, (size_t)nv * std::max<int64_t>(p->cap_S, 1)))) return st;
    if ((st = track(p, &p->v_own, (size_t)nv * std::max<int64_t>(p->cap_S, 1)))) return st;
    if ((st = track(p, &p->v_grad, (size_t)nv * std::max<int64_t>(p->cap_S, 1) * kThetaN))) return st;
    p->nv_slots = nv;
  }
  return CEL_OK;
}

hipError_t stage_selection(cel_plan* p, const std::vector<uint8_t>& m, bool as_class, hipStream_t sm) {
  // the pinned buffers are reused: wait for the previous call's copies out of them
  if (hipEventSynchronize(p->mask_copied) != hipSuccess) return hipErrorUnknown;
  std::memcpy(p->h_mask, m.data(), p->S);
  hipError_t e = hipMemcpyAsync(p->d_mask, p->h_mask, p->S, hipMemcpyHostToDevice, sm);
  if (as_class) {
    const int cls = p->n_colours;
    auto& src = p->class_src[cls];
    auto& pat = p->class_patches[cls];
    auto& tsk = p->class_tasks[cls];
    src.clear();
    pat.clear();
    tsk.clear();
    for (int s = 0; s < p->S; ++s)
      if (m[s]) {
        src.push_back(s);
        for (int i = p->patch_ptr_h[s]; i < p->patch_ptr_h[s + 1]; ++i) pat.push_back(i);
      }
    for (int t : p->order_h)
      if (m[p->patches_h[p->tasks_h[t].patch].src]) tsk.push_back(t);
    int32_t* h = p->h_lists;
    std::memcpy(h, src.data(), src.size() * sizeof(int32_t));
    std::memcpy(h + src.size(), pat.data(), pat.size() * sizeof(int32_t));
    std::memcpy(h + src.size() + pat.size(), tsk.data(), tsk.size() * sizeof(int32_t));
    if (e == hipSuccess && !src.empty())
      e = hipMemcpyAsync(p->d_step_src, h, src.size() * sizeof(int32_t), hipMemcpyHostToDevice, sm);
    if (e == hipSuccess && !pat.empty())
      e = hipMemcpyAsync(p->d_step_patches, h + src.size(), pat.size() * sizeof(int32_t), hipMemcpyHostToDevice, sm);
    if (e == hipSuccess && !tsk.empty())
      e = hipMemcpyAsync(p->d_step_tasks, h + src.size() + pat.size(), tsk.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, sm);
  }
  if (e == hipSuccess) e = hipEventRecord(p->mask_copied, sm);
  return e;
}

cel_status ensure_newton(cel_plan* p) {
  if (p->newton_ready) return CEL_OK;
  cel_status st;
  const size_t S1 = (size_t)std::max<int64_t>(p->cap_S, 1);
  const size_t P1 = (size_t)std::max<int64_t>(p->cap_P, 1), T1 = (size_t)std::max<int64_t>(p->cap_T, 1);
  // (the per-source pixel counts and colours were uploaded with the plan)
  if ((st = track(p, &p->d_theta_trial, S1 * kThetaN)) || (st = track(p, &p->d_pred, S1)) ||
      (st = track(p, &p->d_step_norm, S1)) || (st = track(p, &p->d_trial_active, S1)) ||
      (st = track(p, &p->d_mask, S1)) || (st = track(p, &p->d_counter, 1)) ||
      (st = track(p, &p->d_hslots, T1 * 80)) ||
      (st = track(p, &p->d_step_src, S1)) || (st = track(p, &p->d_step_patches, P1)) ||
      (st = track(p, &p->d_step_tasks, T1)) ||
      (st = track(p, &p->d_hess, S1 * kParamN * kParamN)) ||
      (st = track(p, &p->d_hpart, S1 * kHessParts * kHessPartN)))
    return st;
  if (hipMemset(p->d_trial_active, 0, S1) != hipSuccess) return CEL_EHIP;
  // pinned words, event and stream: the plan's own (after an append), else a kit from a
  // freed plan when one is there
  HostKit k;
  cel_ctx* c = p->ctx;
  if (p->mask_copied) {
    k.h_mask = p->h_mask;
    k.mask_cap = p->mask_cap;
    k.h_lists = p->h_lists;
    k.lists_cap = p->lists_cap;
    k.h_counter = p->h_counter;
    k.h_total = p->h_total;
    k.mask_copied = p->mask_copied;
    k.own_stream = p->own_stream;
  } else if (c && !c->kits.empty()) {
    k = c->kits.back();
    c->kits.pop_back();
  }
  if (k.mask_cap < S1) {
    if (k.h_mask) (void)hipHostFree(k.h_mask);
    k.h_mask = nullptr;
    k.mask_cap = 0;
    if (hipHostMalloc((void**)&k.h_mask, S1, 0) != hipSuccess) return CEL_ENOMEM;
    k.mask_cap = S1;
  }
  const size_t lists = S1 + P1 + T1;
  if (k.lists_cap < lists) {
    if (k.h_lists) (void)hipHostFree(k.h_lists);
    k.h_lists = nullptr;
    k.lists_cap = 0;
    if (hipHostMalloc((void**)&k.h_lists, lists * sizeof(int32_t), 0) != hipSuccess) return CEL_ENOMEM;
    k.lists_cap = lists;
  }
  if (!k.h_counter && hipHostMalloc((void**)&k.h_counter, sizeof(int32_t), 0) != hipSuccess) return CEL_ENOMEM;
  if (!k.h_total && hipHostMalloc((void**)&k.h_total, sizeof(double), 0) != hipSuccess) return CEL_ENOMEM;
  if (!k.mask_copied && hipEventCreate(&k.mask_copied) != hipSuccess) return CEL_EHIP;
  if (!k.own_stream && hipStreamCreate(&k.own_stream) != hipSuccess) return CEL_EHIP;
  p->h_mask = k.h_mask;
  p->mask_cap = k.mask_cap;
  p->h_lists = k.h_lists;
  p->lists_cap = k.lists_cap;
  // the step class (entry n_colours of the class lists), filled by each cel_newton_step
  p->class_src.resize(p->n_colours + 1);
  p->class_patches.resize(p->n_colours + 1);
  p->class_tasks.resize(p->n_colours + 1);
  p->d_class_src.resize(p->n_colours + 1);
  p->d_class_patches.resize(p->n_colours + 1);
  p->d_class_tasks.resize(p->n_colours + 1);
  p->d_class_src[p->n_colours] = p->d_step_src;
  p->d_class_patches[p->n_colours] = p->d_step_patches;
  p->d_class_tasks[p->n_colours] = p->d_step_tasks;
  p->h_counter = k.h_counter;
  p->h_total = k.h_total;
  p->mask_copied = k.mask_copied;
  p->own_stream = k.own_stream;
  p->newton_ready = true;
  return CEL_OK;
}

hipError_t launch_total_after_eval(cel_plan* p, const double* theta, hipStream_t sm) {
  const bool fp64 = p->opt.pixel_fp64 != 0;
  hipError_t e = eval_any(p, theta, nullptr, 0, 1, false, -1, nullptr, sm, true, fp64);
  if (e == hipSuccess) e = launch_total(p->v_own, p->S, p->d_total, sm);
  return e;
}

}  // namespace celmi

// Scratch of cel_elbo_grad_static: one buffer per device for the life of the process, so
// that the entry point allocates nothing.  Host code never uses the array's name as an
// address: each device's copy is at the address hipGetSymbolAddress returns with that
// device current (resolved once per device, at the first cel_create on it).
static __device__ __align__(256) unsigned char scratch[CEL_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device: address of its copy of `scratch`, or null
}  // namespace

// the calling thread's current device must be `device`
static cel_status resolve_static_scratch(int device, int n_devices) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() < n_devices) g_scratch_ptr.resize(n_devices, nullptr);
  if (g_scratch_ptr[device]) return CEL_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CEL_EHIP;
  g_scratch_ptr[device] = ptr;
  return CEL_OK;
}

extern "C" cel_status cel_create(cel_ctx** out, int32_t hip_device, const cel_options* opt) {
  if (!out) return CEL_EINVAL;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess) return CEL_EHIP;
  if (hip_device < 0 || hip_device >= nd) return CEL_EINVAL;
  cel_options o = merge_options(opt);
  resolve_fd_step(o);
  if (!(o.pixels_per_lane == 1 || o.pixels_per_lane == 2 || o.pixels_per_lane == 4)) return CEL_EINVAL;
  if (o.chunk_pixels < 64 || o.chunk_pixels % 64 != 0 || o.chunk_pixels > (1 << 20)) return CEL_EINVAL;
  if (!(o.map_pixels_per_lane == -1 || o.map_pixels_per_lane == 1 || o.map_pixels_per_lane == 2 ||
        o.map_pixels_per_lane == 4 || o.map_pixels_per_lane == 8))
    return CEL_EINVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return CEL_EHIP;
  if (resolve_static_scratch(hip_device, nd) != CEL_OK) return CEL_EHIP;
  int32_t* err = nullptr;
  if (hipMalloc((void**)&err, sizeof(int32_t)) != hipSuccess) return CEL_ENOMEM;
  if (hipMemset(err, 0, sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(err);
    return CEL_EHIP;
  }
  double* table = nullptr;
  if (hipMalloc((void**)&table, sizeof(double) * kCountTable) != hipSuccess) {
    (void)hipFree(err);
    return CEL_ENOMEM;
  }
  if (launch_count_table(table, nullptr) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
    (void)hipFree(table);
    (void)hipFree(err);
    return CEL_EHIP;
  }
  cel_ctx* c = new cel_ctx;
  c->device = hip_device;
  c->opt = o;
  c->d_err = err;
  c->d_ctable = table;
  *out = c;
  return CEL_OK;
}

extern "C" void cel_destroy(cel_ctx* ctx) { ctx_release(ctx); }

extern "C" cel_status cel_last_device_error(cel_ctx* ctx, int32_t* code) {
  if (!ctx || !code) return CEL_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return CEL_EHIP;
  int32_t v = 0;
  if (hipMemcpy(&v, ctx->d_err, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return CEL_EHIP;
  if (hipMemset(ctx->d_err, 0, sizeof(int32_t)) != hipSuccess) return CEL_EHIP;
  *code = v;
  return CEL_OK;
}

extern "C" void cel_plan_free(cel_plan* plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->device);
  plan_release(plan);
}

// The plan's work items at its chunk size (opt.chunk_pixels): the items of every patch, the
// patches' item ranges, the launch order, the moment-map items over the patches' overlap
// boxes and the per-colour item lists.  Host tables only.
namespace celmi {
cel_status build_tiling(cel_plan* p) {
  // work items: runs of chunk pixels per patch (patch-major), launch order by cost
  // Cost of a work item: pixels x (1 + neighbour patches / 2), kept as the integer
  // pixels x (2 + neighbour patches); the order is by decreasing cost, ties by item id
  // (keys: inverted cost above the id).
  const int CH = p->opt.chunk_pixels;
  int64_t n_items = 0;
  for (int i = 0; i < p->P; ++i) n_items += ((int64_t)p->patches_h[i].w * p->patches_h[i].h + CH - 1) / CH;
  if (n_items > (int64_t)1 << 30) return CEL_EUNSUPPORTED;
  p->tasks_h.clear();
  p->tasks_h.reserve(n_items);
  std::vector<uint64_t> keys;
  keys.reserve(n_items);
  for (int i = 0; i < p->P; ++i) {
    DPatch& d = p->patches_h[i];
    const int n = d.w * d.h;
    d.task_begin = (int)p->tasks_h.size();
    for (int b = 0; b < n; b += CH) {
      DTask t;
      t.patch = i;
      t.pix_begin = b;
      t.pix_end = std::min(n, b + CH);
      t.pad = 0;
      const uint64_t c = (uint64_t)(t.pix_end - t.pix_begin) * (uint64_t)(2 + (d.nbr_end - d.nbr_begin));
      const uint64_t inv = 0xffffffffull - std::min<uint64_t>(c, 0xffffffffull);
      keys.push_back((inv << 32) | (uint64_t)p->tasks_h.size());
      p->tasks_h.push_back(t);
    }
    d.task_end = (int)p->tasks_h.size();
  }
  p->n_tasks = (int64_t)p->tasks_h.size();
  // stable LSD radix sort on the inverted cost (the ids are generated in ascending order)
  {
    std::vector<uint64_t> tmp(keys.size());
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = 32 + 8 * pass;
      size_t count[257] = {0};
      for (uint64_t k : keys) ++count[((k >> shift) & 0xff) + 1];
      for (int b = 0; b < 256; ++b) count[b + 1] += count[b];
      for (uint64_t k : keys) tmp[count[(k >> shift) & 0xff]++] = k;
      keys.swap(tmp);
    }
  }
  p->order_h.resize(p->n_tasks);
  for (int64_t i = 0; i < p->n_tasks; ++i) p->order_h[i] = (int32_t)(keys[i] & 0xffffffffull);
  // the moment maps are read only where another source's patch overlaps: the map work
  // items cover each patch's overlap box (the bounding box of its intersections with its
  // neighbours' rectangles) in runs of at most CH pixels, row-major within the box, larger
  // runs first (a patch's full runs stay together)
  p->map_tasks_h.clear();
  for (int i = 0; i < p->P; ++i) {
    const DPatch& d = p->patches_h[i];
    int bx0 = d.w, bx1 = 0, by0 = d.h, by1 = 0;
    for (int nb = d.nbr_begin; nb < d.nbr_end; ++nb) {
      const DPatch& q = p->patches_h[p->nbr_idx_h[nb]];
      const int xa = std::max(q.x0 - d.x0, 0), xb = std::min(q.x0 + q.w - d.x0, d.w);
      const int ya = std::max(q.y0 - d.y0, 0), yb = std::min(q.y0 + q.h - d.y0, d.h);
      if (xb <= xa || yb <= ya) continue;
      bx0 = std::min(bx0, xa);
      bx1 = std::max(bx1, xb);
      by0 = std::min(by0, ya);
      by1 = std::max(by1, yb);
    }
    if (bx1 <= bx0 || by1 <= by0) continue;
    const int bw = bx1 - bx0, n = bw * (by1 - by0);
    for (int b = 0; b < n; b += CH) {
      DMapTask m;
      std::memset(&m, 0, sizeof(m));
      m.patch = i;
      m.pix_begin = b;
      m.pix_end = std::min(n, b + CH);
      m.x0 = bx0;
      m.y0 = by0;
      m.w = bw;
      p->map_tasks_h.push_back(m);
    }
  }
  std::stable_sort(p->map_tasks_h.begin(), p->map_tasks_h.end(), [](const DMapTask& u, const DMapTask& v) {
    return u.pix_end - u.pix_begin > v.pix_end - v.pix_begin;
  });
  // per-colour work-item lists (for masked launches), in launch order
  p->class_tasks.resize(std::max<size_t>(p->class_tasks.size(), (size_t)p->n_colours));
  for (int c = 0; c < p->n_colours; ++c) p->class_tasks[c].clear();
  for (int i : p->order_h) {
    const int c = p->colour[p->patches_h[p->tasks_h[i].patch].src];
    p->class_tasks[c].push_back(i);
  }
  return CEL_OK;
}
}  // namespace celmi

extern "C" cel_status cel_prepare(cel_ctx* ctx, const cel_problem* pr, cel_plan** out, void* stream) {
  if (!ctx || !out) return CEL_EINVAL;
  *out = nullptr;
  cel_status st = validate(pr);
  if (st) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  cel_plan* p = new cel_plan;
  p->device = ctx->device;
  p->opt = ctx->opt;
  p->d_err = ctx->d_err;
  p->ctx = ctx;
  ++ctx->refs;
  const int S = pr->n_sources, N = pr->n_images, P = pr->n_patches;
  p->S = S;
  p->N = N;
  p->P = P;
  p->images_h.assign(pr->images, pr->images + N);
  // patches: packed offsets in our own (count, sky) array, CSR per source
  p->patches_h.resize(P);
  p->patch_ptr_h.assign(S + 1, 0);
  int64_t off = 0;
  for (int i = 0; i < P; ++i) {
    const cel_patch& q = pr->patches[i];
    DPatch d;
    d.src = q.src; d.img = q.img; d.x0 = q.x0; d.y0 = q.y0; d.w = q.w; d.h = q.h;
    d.off = off;
    off += (int64_t)q.w * q.h;
    p->patches_h[i] = d;
    p->patch_ptr_h[q.src + 1]++;
  }
  p->n_units = off;
  for (int s = 0; s < S; ++s) p->patch_ptr_h[s + 1] += p->patch_ptr_h[s];
  // neighbour patches: same image, other source, intersecting rectangles (sweep over x0);
  // the pairs are counted per patch and scattered into the CSR list, then each patch's
  // (short) list is sorted ascending
  {
    // (image, x0, id) order by one integer sort of packed keys (image < 2^20, x0 < 2^20 and
    // id < 2^24, checked by validate), then the rectangles in that order, contiguous
    struct Rect {
      int32_t img, x0, x1, y0, y1, src, id;
    };
    std::vector<uint64_t> key(P);
    for (int i = 0; i < P; ++i) {
      const DPatch& d = p->patches_h[i];
      key[i] = ((uint64_t)d.img << 44) | ((uint64_t)d.x0 << 24) | (uint64_t)i;
    }
    std::sort(key.begin(), key.end());
    std::vector<Rect> r(P);
    for (int i = 0; i < P; ++i) {
      const int id = (int)(key[i] & 0xffffffu);
      const DPatch& d = p->patches_h[id];
      r[i] = Rect{d.img, d.x0, d.x0 + d.w, d.y0, d.y0 + d.h, d.src, id};
    }
    std::vector<int2> pairs;
    std::vector<int> deg(P + 1, 0);
    for (int ia = 0; ia < P; ++ia) {
      const Rect& A = r[ia];
      for (int ib = ia + 1; ib < P; ++ib) {
        const Rect& B = r[ib];
        if (B.img != A.img || B.x0 >= A.x1) break;
        if (B.y0 < A.y1 && A.y0 < B.y1 && A.src != B.src) {
          pairs.push_back(make_int2(A.id, B.id));
          ++deg[A.id];
          ++deg[B.id];
        }
      }
    }
    int e = 0;
    for (int i = 0; i < P; ++i) {
      p->patches_h[i].nbr_begin = p->patches_h[i].nbr_end = e;
      e += deg[i];
    }
    p->nbr_idx_h.resize(e);
    for (const int2& q : pairs) {
      p->nbr_idx_h[p->patches_h[q.x].nbr_end++] = q.y;
      p->nbr_idx_h[p->patches_h[q.y].nbr_end++] = q.x;
    }
    for (int i = 0; i < P; ++i)
      std::sort(p->nbr_idx_h.begin() + p->patches_h[i].nbr_begin, p->nbr_idx_h.begin() + p->patches_h[i].nbr_end);
  }
  // source overlap graph (neighbour patches' sources, without repeats) and greedy colouring
  // (ascending id, smallest free colour)
  p->adj.assign(S, {});
  for (int i = 0; i < P; ++i)
    for (int e = p->patches_h[i].nbr_begin; e < p->patches_h[i].nbr_end; ++e)
      p->adj[p->patches_h[i].src].push_back(p->patches_h[p->nbr_idx_h[e]].src);
  for (auto& a : p->adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  p->colour.assign(S, -1);
  p->n_colours = 0;
  {
    std::vector<char> used;
    for (int s = 0; s < S; ++s) {
      used.assign(p->adj[s].size() + 1, 0);
      for (int t : p->adj[s])
        if (p->colour[t] >= 0 && p->colour[t] < (int)used.size()) used[p->colour[t]] = 1;
      int c = 0;
      while (used[c]) ++c;
      p->colour[s] = c;
      p->n_colours = std::max(p->n_colours, c + 1);
    }
  }
  p->class_patches.assign(p->n_colours, {});
  p->class_src.assign(p->n_colours, {});
  for (int s = 0; s < S; ++s) {
    const int c = p->colour[s];
    p->class_src[c].push_back(s);
    for (int i = p->patch_ptr_h[s]; i < p->patch_ptr_h[s + 1]; ++i) p->class_patches[c].push_back(i);
  }
  if ((st = build_tiling(p))) {
    plan_release(p);
    return st;
  }
  p->cap_S = S;
  p->cap_P = P;
  p->cap_T = p->n_tasks;
  p->cap_U = p->n_units;
  // prior tables
  {
    const cel_prior& pp = *pr->prior;
    DPrior d;
    std::memset(&d, 0, sizeof(d));
    d.logit_a = std::log(pp.star_prob / (1 - pp.star_prob));
    d.log_a = std::log(pp.star_prob);
    d.log_1ma = std::log1p(-pp.star_prob);
    for (int i = 0; i < 2; ++i) {
      d.r[i][0] = pp.r[i][0];
      d.r[i][1] = pp.r[i][1];
      for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) {
        d.c_logw[i][j] = pp.c_w[i][j] > 0 ? std::log(pp.c_w[i][j]) : -1e300;
        for (int k = 0; k < 4; ++k) d.c_mean[i][j][k] = pp.c_mean[i][j][k];
        double ld = 0;
        if (pp.c_w[i][j] > 0) spd_inverse4(pp.c_cov[i][j], d.c_prec[i][j], &ld);
        d.c_logdet[i][j] = ld;
      }
    }
    d.radius[0] = pp.radius[0];
    d.radius[1] = pp.radius[1];
    d.profile[0] = pp.profile[0];
    d.profile[1] = pp.profile[1];
    d.axis[0] = pp.axis[0];
    d.axis[1] = pp.axis[1];
    d.lbeta_profile = std::lgamma(pp.profile[0]) + std::lgamma(pp.profile[1]) - std::lgamma(pp.profile[0] + pp.profile[1]);
    d.lbeta_axis = std::lgamma(pp.axis[0]) + std::lgamma(pp.axis[1]) - std::lgamma(pp.axis[0] + pp.axis[1]);
    p->prior_h = d;
  }
  {
    const cel_profiles& pf = *pr->profiles;
    DProfiles d;
    std::memset(&d, 0, sizeof(d));
    d.n_exp = pf.n_exp;
    d.n_dev = pf.n_dev;
    for (int j = 0; j < pf.n_exp; ++j) { d.alpha[j] = pf.exp_alpha[j]; d.tau[j] = pf.exp_tau[j]; }
    for (int j = 0; j < pf.n_dev; ++j) { d.alpha[pf.n_exp + j] = pf.dev_alpha[j]; d.tau[pf.n_exp + j] = pf.dev_tau[j]; }
    p->prof_h = d;
    p->nexp = pf.n_exp;
    p->ndev = pf.n_dev;
  }
  std::vector<int32_t> npsf(std::max(N, 1), 1);
  for (int n = 0; n < N; ++n) npsf[n] = pr->images[n].n_psf;
  std::vector<int64_t> user_off(std::max(P, 1), 0);
  for (int i = 0; i < P; ++i) user_off[i] = pr->patches[i].pix_off;
  std::vector<double> knots(pr->sky_knots, pr->sky_knots + pr->n_sky_knots);
  std::vector<cel_image> imgs = p->images_h;
  std::vector<DPrior> prior1(1, p->prior_h);
  std::vector<DProfiles> prof1(1, p->prof_h);
  int64_t* d_user_off = nullptr;
  double* d_knots = nullptr;
  // the plan's tables and lists, the per-colour lists included, in one transfer
  UploadPack pk;
  pk.add(&p->d_patches, p->patches_h);
  pk.add(&p->d_images, imgs);
  pk.add(&p->d_nbr, p->nbr_idx_h);
  pk.add(&p->d_tasks, p->tasks_h);
  pk.add(&p->d_order, p->order_h);
  pk.add(&p->d_map_tasks, p->map_tasks_h);
  pk.add(&p->d_patch_ptr, p->patch_ptr_h);
  pk.add(&p->d_npsf, npsf);
  pk.add(&p->d_prior, prior1);
  pk.add(&p->d_prof, prof1);
  pk.add(&d_user_off, user_off);
  pk.add(&d_knots, knots);
  std::vector<double> ppsf;
  if (pr->patch_psf && P > 0) {
    ppsf.assign(pr->patch_psf, pr->patch_psf + (size_t)P * kMaxPsf * 6);
    pk.add(&p->d_patch_psf, ppsf);
  }
  // per-source active pixel counts and colours (read by the Newton steps)
  std::vector<double> npix(std::max(S, 1), 0.0);
  for (int i = 0; i < P; ++i) npix[p->patches_h[i].src] += (double)p->patches_h[i].w * p->patches_h[i].h;
  std::vector<int32_t> col(std::max(S, 1), 0);
  for (int s = 0; s < S; ++s) col[s] = p->colour[s];
  pk.add(&p->d_npix, npix);
  pk.add(&p->d_colour, col);
  p->d_class_patches.assign(p->n_colours, nullptr);
  p->d_class_tasks.assign(p->n_colours, nullptr);
  p->d_class_src.assign(p->n_colours, nullptr);
  for (int c = 0; c < p->n_colours; ++c) {
    pk.add(&p->d_class_patches[c], p->class_patches[c]);
    pk.add(&p->d_class_tasks[c], p->class_tasks[c]);
    pk.add(&p->d_class_src[c], p->class_src[c]);
  }
  if ((st = upload_pack(p, pk, sm)) || (st = track(p, &p->d_xs, (size_t)std::max<int64_t>(p->n_units, 1))) ||
      (st = track(p, &p->d_pixconst, (size_t)2 * std::max(P, 1))) || (st = track(p, &p->d_skymin, (size_t)std::max(P, 1))) || (st = track(p, &p->d_total, 1)) ||
      (st = ensure_variants(p, 1, p->opt.pixel_fp64 != 0))) {
    plan_release(p);
    return st;
  }
  if ((st = track(p, &p->d_maps, (size_t)std::max<int64_t>(p->n_units, 1))) ||
      ((p->opt.pixel_fp64 || p->opt.hessian_fp64) &&
       ((st = track(p, &p->d_xs64, (size_t)std::max<int64_t>(p->n_units, 1))) ||
        (st = track(p, &p->d_maps64, (size_t)std::max<int64_t>(p->n_units, 1)))))) {
    plan_release(p);
    return st;
  }
  hipError_t e = launch_pixels(p->d_patches, p->d_images, d_knots, pr->pixels, d_user_off, p->d_xs, p->d_xs64, P, sm);
  if (e == hipSuccess)
    e = launch_pixconst(p->d_patches, p->d_nbr, p->d_xs, ctx->d_ctable, p->d_pixconst, p->d_skymin, P, sm);
  if (e == hipSuccess) e = hipStreamSynchronize(sm);
  if (e != hipSuccess) {
    plan_release(p);
    return CEL_EHIP;
  }
  *out = p;
  return CEL_OK;
}

extern "C" cel_status cel_plan_info(const cel_plan* plan, int64_t* n_units, int32_t* n_colours, int32_t* colours,
                                    int64_t* n_work_items, int64_t* device_bytes) {
  if (!plan) return CEL_EINVAL;
  if (device_bytes) {
    int64_t b = 0;
    for (const auto& blk : plan->allocs) b += (int64_t)blk.bytes;
    *device_bytes = b;
  }
  if (n_units) *n_units = plan->n_units;
  if (n_colours) *n_colours = plan->n_colours;
  if (n_work_items) *n_work_items = plan->n_tasks;
  if (colours)
    for (int s = 0; s < plan->S; ++s) colours[s] = plan->colour[s];
  return CEL_OK;
}

namespace celmi {

template <typename T>
static hipError_t launch_maps_t(cel_plan* p, const Table<T>* tables, hipStream_t sm) {
  MapArgs ma;
  std::memset(&ma, 0, sizeof(ma));
  ma.tasks = p->d_map_tasks;
  ma.patches = p->d_patches;
  ma.base = tables;
  ma.maps = sizeof(T) == 8 ? (void*)p->d_maps64 : (void*)p->d_maps;
  ma.img_npsf = p->d_npsf;
  return launch_maps<T>(ma, p->nexp, p->ndev, p->opt.map_pixels_per_lane, (int)p->map_tasks_h.size(), sm);
}

// Enqueue prep + fused + finalize for `nv` variants starting at variant v0 over either all
// sources (cls < 0) or one colour class, with optional active mask.  Outputs go to the
// plan's per-variant arrays.
constexpr int kPointPixelsPerLane = 4;

template <typename T>
static hipError_t enqueue_eval(cel_plan* p, const double* theta, const double* theta_trial, int v0, int nv,
                               bool grad, int cls, const uint8_t* active, hipStream_t sm, bool prep_base,
                               double* local_out, double* grad_out, int64_t theta_vstride = 0,
                               const uint8_t* active_v = nullptr) {
  // theta_vstride > 0: likelihood mode -- variant v's parameters at theta + v * theta_vstride,
  // no differences, no KL, the pixel sums of variant v to local_out + v * S
  const bool point = theta_vstride > 0;
  Table<T>* tables = reinterpret_cast<Table<T>*>(sizeof(T) == 8 ? (void*)p->tables_d : (void*)p->tables_f);
  hipError_t e = hipSuccess;
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.theta = theta;
  pa.theta_trial = theta_trial;
  pa.fd_step = p->opt.fd_step;
  pa.patches = p->d_patches;
  pa.images = p->d_images;
  pa.prof = p->d_prof;
  pa.tables = tables;
  pa.n_patches = p->P;
  pa.trial_variant = p->trial_variant;
  pa.fd = point ? 0 : p->fd_mode;
  pa.sky_min = p->d_skymin;
  pa.patch_psf = p->d_patch_psf;
  pa.records = p->opt.map_pixels_per_lane == -1 ? kRecRuns : 0;
  pa.theta_vstride = theta_vstride;
  pa.active_v = active_v;   // (launch variant, source) pairs to evaluate: the likelihood pass
  pa.active_v_stride = p->S;
  phase_mark(p, 0, sm);
  if (prep_base) {   // variant 0 of every source and its moment maps (neighbours read these)
    pa.variant0 = 0;
    e = launch_prep_tables<T>(pa, p->P, 1, sm);
    if (e != hipSuccess) return e;
    phase_mark(p, 1, sm);
    e = launch_maps_t<T>(p, tables, sm);
    if (e != hipSuccess) return e;
  }
  int n_items = (int)p->n_tasks;
  const int32_t* order = p->d_order;
  if (cls >= 0) {
    pa.patch_list = p->d_class_patches[cls];
    n_items = (int)p->class_tasks[cls].size();
    order = p->d_class_tasks[cls];
  }
  pa.active = active;
  const int vstart = (v0 == 0 && prep_base) ? 1 : 0;   // variant 0 already prepared
  if (nv - vstart > 0) {
    pa.variant0 = v0 + vstart;
    const int np = cls >= 0 ? (int)p->class_patches[cls].size() : p->P;
    e = launch_prep_tables<T>(pa, np, nv - vstart, sm);
    if (e != hipSuccess) return e;
  }
  phase_mark(p, 2, sm);
  FusedArgs<T> fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.tasks = p->d_tasks;
  fa.order = order;
  fa.order_offset = 0;
  fa.patches = p->d_patches;
  fa.nbr_idx = p->d_nbr;
  fa.base = tables;
  fa.own = tables;
  fa.variant_stride = p->P;
  fa.xs = sizeof(T) == 8 ? (const void*)p->d_xs64 : (const void*)p->d_xs;
  fa.maps = sizeof(T) == 8 ? (const void*)p->d_maps64 : (const void*)p->d_maps;
  fa.slots = p->slots + (int64_t)v0 * p->n_tasks * kSlots;
  fa.slot_variant_stride = p->n_tasks * kSlots;
  fa.active = active;
  fa.variant0 = v0;
  fa.img_npsf = p->d_npsf;
  fa.active_v = active_v;
  fa.active_v_stride = p->S;
  // the likelihood pass (values only, often one type per candidate) takes 4 pixels per lane
  // whatever the plan's setting: more independent work per wavefront for thin candidates
  // (10.2 ms per 56 x 1000 candidates against 12.1 at 2 and 10.8 at 8)
  const int ppl = point ? kPointPixelsPerLane : p->opt.pixels_per_lane;
  e = launch_fused<T>(fa, p->nexp, p->ndev, ppl, grad, n_items, nv, sm);
  if (e != hipSuccess) return e;
  phase_mark(p, 3, sm);
  FinalizeArgs fz;
  std::memset(&fz, 0, sizeof(fz));
  fz.n_jobs = p->S;
  fz.variant0 = v0;
  fz.active = active;
  fz.theta = theta;
  fz.theta_trial = theta_trial;
  fz.fd_step = p->opt.fd_step;
  fz.slots = p->slots + (int64_t)v0 * p->n_tasks * kSlots;
  fz.slot_variant_stride = p->n_tasks * kSlots;
  fz.patch_ptr = p->d_patch_ptr;
  fz.patches = p->d_patches;
  fz.pix_const = p->d_pixconst;
  fz.err = p->d_err;
  fz.images = p->d_images;
  fz.prior = p->d_prior;
  fz.want_grad = grad ? 1 : 0;
  const bool direct = (v0 == 0 && nv == 1) || point;
  fz.local = direct && local_out ? local_out : p->v_local + (int64_t)v0 * p->S;
  fz.own = p->v_own + (int64_t)v0 * p->S;
  fz.grad = direct && grad_out ? grad_out : p->v_grad + (int64_t)v0 * p->S * kThetaN;
  fz.out_variant_stride = p->S;
  fz.trial_variant = p->trial_variant;
  fz.fd = point ? 0 : p->fd_mode;
  fz.theta_vstride = theta_vstride;
  fz.no_kl = point ? 1 : 0;
  fz.active_v = active_v;
  fz.active_v_stride = p->S;
  if (point) fz.err = nullptr;   // a candidate's non-finite likelihood is a result, not a fault
  if (cls >= 0) {
    // jobs = members of the class
    fz.n_jobs = (int)p->class_src[cls].size();
    fz.job_src = p->d_class_src[cls];
  }
  return launch_finalize(fz, nv, sm);
}

template <typename T>
static hipError_t plain_eval_t(cel_plan* p, const double* theta, hipStream_t sm) {
  Table<T>* tables = reinterpret_cast<Table<T>*>(sizeof(T) == 8 ? (void*)p->tables_d : (void*)p->tables_f);
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.theta = theta;
  pa.fd_step = p->opt.fd_step;
  pa.patches = p->d_patches;
  pa.images = p->d_images;
  pa.prof = p->d_prof;
  pa.tables = tables;
  pa.n_patches = p->P;
  pa.trial_variant = p->trial_variant;
  pa.fd = p->fd_mode;
  pa.sky_min = p->d_skymin;
  pa.patch_psf = p->d_patch_psf;
  pa.records = p->opt.map_pixels_per_lane == -1 ? kRecRuns : 0;
  hipError_t e = launch_prep_tables<T>(pa, p->P, 1, sm);
  if (e == hipSuccess) e = launch_maps_t<T>(p, tables, sm);
  FusedArgs<T> fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.tasks = p->d_tasks;
  fa.order = nullptr;
  fa.patches = p->d_patches;
  fa.nbr_idx = p->d_nbr;
  fa.base = tables;
  fa.own = tables;
  fa.variant_stride = p->P;
  fa.xs = sizeof(T) == 8 ? (const void*)p->d_xs64 : (const void*)p->d_xs;
  fa.maps = sizeof(T) == 8 ? (const void*)p->d_maps64 : (const void*)p->d_maps;
  fa.slots = p->slots;
  fa.slot_variant_stride = p->n_tasks * kSlots;
  fa.img_npsf = p->d_npsf;
  FinalizeArgs fz;
  std::memset(&fz, 0, sizeof(fz));
  fz.n_jobs = 1;
  fz.theta = theta;
  fz.fd_step = p->opt.fd_step;
  fz.slots = p->slots;
  fz.slot_variant_stride = p->n_tasks * kSlots;
  fz.patch_ptr = p->d_patch_ptr;
  fz.patches = p->d_patches;
  fz.pix_const = p->d_pixconst;
  fz.err = p->d_err;
  fz.images = p->d_images;
  fz.prior = p->d_prior;
  fz.want_grad = 1;
  fz.trial_variant = p->trial_variant;
  fz.fd = p->fd_mode;
  fz.local = p->v_local;
  fz.own = p->v_own;
  fz.grad = p->v_grad;
  fz.out_variant_stride = p->S;
  for (int s = 0; s < p->S && e == hipSuccess; ++s) {
    const int pb = p->patch_ptr_h[s], pe = p->patch_ptr_h[s + 1];
    if (pe > pb) {
      const int tb = p->patches_h[pb].task_begin, te = p->patches_h[pe - 1].task_end;
      fa.order_offset = tb;
      e = launch_fused<T>(fa, p->nexp, p->ndev, p->opt.pixels_per_lane, true, te - tb, 1, sm);
    }
    fz.src_offset = s;
    if (e == hipSuccess) e = launch_finalize(fz, 1, sm);
  }
  return e;
}

hipError_t plain_eval(cel_plan* p, const double* theta, hipStream_t sm, bool fp64) {
  return fp64 ? plain_eval_t<double>(p, theta, sm) : plain_eval_t<float>(p, theta, sm);
}

template <typename T>
static hipError_t prep_base_t(cel_plan* p, const double* theta, hipStream_t sm, bool hess) {
  Table<T>* tables = reinterpret_cast<Table<T>*>(sizeof(T) == 8 ? (void*)p->tables_d : (void*)p->tables_f);
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.theta = theta;
  pa.fd_step = p->opt.fd_step;
  pa.patches = p->d_patches;
  pa.images = p->d_images;
  pa.prof = p->d_prof;
  pa.tables = tables;
  pa.n_patches = p->P;
  pa.trial_variant = p->trial_variant;
  pa.fd = p->fd_mode;
  pa.sky_min = p->d_skymin;
  pa.patch_psf = p->d_patch_psf;
  pa.records = (p->opt.map_pixels_per_lane == -1 ? kRecRuns : 0) | (hess ? kRecHessian : 0);
  hipError_t e = launch_prep_tables<T>(pa, p->P, 1, sm);
  if (e == hipSuccess) e = launch_maps_t<T>(p, tables, sm);
  return e;
}

hipError_t prep_base(cel_plan* p, const double* theta, hipStream_t sm, bool fp64, bool hess) {
  return fp64 ? prep_base_t<double>(p, theta, sm, hess) : prep_base_t<float>(p, theta, sm, hess);
}

template <typename T>
static hipError_t prep_class_t(cel_plan* p, const double* theta, int cls, const uint8_t* active, hipStream_t sm,
                               bool hess) {
  const int np = (int)p->class_patches[cls].size();
  if (np == 0) return hipSuccess;
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.theta = theta;
  pa.fd_step = p->opt.fd_step;
  pa.patch_list = p->d_class_patches[cls];
  pa.patches = p->d_patches;
  pa.images = p->d_images;
  pa.prof = p->d_prof;
  pa.tables = sizeof(T) == 8 ? (void*)p->tables_d : (void*)p->tables_f;
  pa.n_patches = p->P;
  pa.active = active;
  pa.trial_variant = p->trial_variant;
  pa.fd = p->fd_mode;
  pa.sky_min = p->d_skymin;
  pa.patch_psf = p->d_patch_psf;
  pa.records = (p->opt.map_pixels_per_lane == -1 ? kRecRuns : 0) | (hess ? kRecHessian : 0);
  return launch_prep_tables<T>(pa, np, 1, sm);
}

hipError_t prep_class(cel_plan* p, const double* theta, int cls, const uint8_t* active, hipStream_t sm, bool fp64,
                      bool hess) {
  return fp64 ? prep_class_t<double>(p, theta, cls, active, sm, hess)
              : prep_class_t<float>(p, theta, cls, active, sm, hess);
}

hipError_t eval_any(cel_plan* p, const double* theta, const double* theta_trial, int v0, int nv, bool grad, int cls,
                    const uint8_t* active, hipStream_t sm, bool prep_base, bool fp64, double* local_out,
                    double* grad_out) {
  return fp64 ? enqueue_eval<double>(p, theta, theta_trial, v0, nv, grad, cls, active, sm, prep_base, local_out,
                                     grad_out)
              : enqueue_eval<float>(p, theta, theta_trial, v0, nv, grad, cls, active, sm, prep_base, local_out,
                                    grad_out);
}

}  // namespace celmi

static cel_status eval_common(cel_ctx* ctx, const cel_plan* cplan, const double* theta, double* elbo_total,
                              double* elbo_local, double* grad, void* stream, bool want_grad) {
  if (!ctx || !cplan || (!theta && cplan->S > 0)) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  const bool fp64 = p->opt.pixel_fp64 != 0;
  cel_status st = ensure_variants(p, 1, fp64);
  if (st) return st;
  p->marking = true;
  // the finalisation writes the caller's local objectives and gradients directly
  hipError_t e = eval_any(p, theta, nullptr, 0, 1, want_grad, -1, nullptr, sm, true, fp64, elbo_local,
                          want_grad ? grad : nullptr);
  if (e == hipSuccess && elbo_total) e = launch_total(p->v_own, p->S, elbo_total, sm);
  phase_mark(p, 4, sm);
  p->marking = false;
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

// cel_elbo_grad with its per-call scratch in the static buffer: the component tables, the
// neighbour moment maps, the slot rows and the per-source sums are carved from `scratch`
// (256-byte aligned parts) instead of the plan's own blocks; the kernels are the same.
// Every part is written in full by the evaluation before it is read, so nothing is cleared.
extern "C" cel_status cel_elbo_grad_static(cel_ctx* ctx, const cel_plan* cplan, const double* theta,
                                           double* elbo_total, double* elbo_local, double* grad, void* stream) {
  if (!ctx || !cplan || (!theta && cplan->S > 0)) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (p->device != ctx->device) return CEL_EINVAL;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (p->device < (int)g_scratch_ptr.size()) base = g_scratch_ptr[p->device];
  }
  if (!base) return CEL_EHIP;   // cel_create resolves it; a context on this device exists
  const bool fp64 = p->opt.pixel_fp64 != 0;
  const size_t align = 256;
  auto up = [&](size_t b) { return (b + align - 1) / align * align; };
  const size_t P1 = (size_t)std::max(p->P, 1), S1 = (size_t)std::max(p->S, 1);
  const size_t b_tables = up(P1 * (fp64 ? sizeof(Table<double>) : sizeof(Table<float>)));
  const size_t b_maps = up((size_t)std::max<int64_t>(p->n_units, 1) * (fp64 ? sizeof(double2) : sizeof(float2)));
  const size_t b_slots = up((size_t)std::max<int64_t>(p->n_tasks, 1) * kSlots * sizeof(double));
  const size_t b_src = up(S1 * sizeof(double));
  const size_t b_grad = up(S1 * kThetaN * sizeof(double));
  const size_t need = b_tables + b_maps + b_slots + 2 * b_src + b_grad;
  if (need > (size_t)CEL_STATIC_SCRATCH_BYTES) return CEL_ESCRATCH;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  unsigned char* q = static_cast<unsigned char*>(base);
  void* tables = q;
  void* maps = q + b_tables;
  double* slots = reinterpret_cast<double*>(q + b_tables + b_maps);
  double* own = reinterpret_cast<double*>(q + b_tables + b_maps + b_slots);
  double* local = reinterpret_cast<double*>(q + b_tables + b_maps + b_slots + b_src);
  double* gscr = reinterpret_cast<double*>(q + b_tables + b_maps + b_slots + 2 * b_src);
  // the plan's scratch pointers point into the static buffer while the launches are enqueued
  Table<float>* s_tf = p->tables_f;
  Table<double>* s_td = p->tables_d;
  float2* s_mf = p->d_maps;
  double2* s_md = p->d_maps64;
  double *s_slots = p->slots, *s_own = p->v_own, *s_local = p->v_local, *s_grad = p->v_grad;
  if (fp64) {
    p->tables_d = static_cast<Table<double>*>(tables);
    p->d_maps64 = static_cast<double2*>(maps);
  } else {
    p->tables_f = static_cast<Table<float>*>(tables);
    p->d_maps = static_cast<float2*>(maps);
  }
  p->slots = slots;
  p->v_own = own;
  p->v_local = local;
  p->v_grad = gscr;
  const bool marking = p->marking;
  p->marking = false;   // no timing events: creating them may allocate
  hipStream_t sm = (hipStream_t)stream;
  hipError_t e = eval_any(p, theta, nullptr, 0, 1, true, -1, nullptr, sm, true, fp64, elbo_local, grad);
  if (e == hipSuccess && elbo_total) e = launch_total(p->v_own, p->S, elbo_total, sm);
  p->tables_f = s_tf;
  p->tables_d = s_td;
  p->d_maps = s_mf;
  p->d_maps64 = s_md;
  p->slots = s_slots;
  p->v_own = s_own;
  p->v_local = s_local;
  p->v_grad = s_grad;
  p->marking = marking;
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

extern "C" cel_status cel_elbo_eval(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                                    double* elbo_local, void* stream) {
  return eval_common(ctx, plan, theta, elbo_total, elbo_local, nullptr, stream, false);
}

extern "C" cel_status cel_elbo_grad(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                                    double* elbo_local, double* grad, void* stream) {
  return eval_common(ctx, plan, theta, elbo_total, elbo_local, grad, stream, true);
}

// Plain form: the same kernels, one launch of the pixel kernel and of the finalisation per
// source, in source order, with work items in patch order.
extern "C" cel_status cel_elbo_grad_plain(cel_ctx* ctx, const cel_plan* cplan, const double* theta,
                                          double* elbo_total, double* elbo_local, double* grad, void* stream) {
  if (!ctx || !cplan || (!theta && cplan->S > 0)) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  const bool fp64 = p->opt.pixel_fp64 != 0;
  cel_status st = ensure_variants(p, 1, fp64);
  if (st) return st;
  hipError_t e = plain_eval(p, theta, sm, fp64);
  if (e == hipSuccess && elbo_total) e = launch_total(p->v_own, p->S, elbo_total, sm);
  if (e == hipSuccess && elbo_local && p->S > 0)
    e = hipMemcpyAsync(elbo_local, p->v_local, sizeof(double) * p->S, hipMemcpyDeviceToDevice, sm);
  if (e == hipSuccess && grad && p->S > 0)
    e = hipMemcpyAsync(grad, p->v_grad, sizeof(double) * p->S * kThetaN, hipMemcpyDeviceToDevice, sm);
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

// Exact Poisson log-likelihood at point values (Section 3.1's target p(x | w_s, a_s, z_{-s})):
// the other sources at z_fixed give the neighbour maps once; each chunk of candidates is a
// set of variants of the objective's pixel pass over the selected sources' work items.
namespace celmi {

cel_status point_setup(cel_plan* p, const double* z_fixed, const std::vector<uint8_t>& m, int chunk, hipStream_t sm) {
  const bool fp64 = p->opt.pixel_fp64 != 0;
  const int S = p->S;
  cel_status st = ensure_variants(p, chunk, fp64);
  if (st == CEL_OK) st = ensure_newton(p);
  if (st == CEL_OK && p->pt_cap < chunk) {
    if ((st = track(p, &p->d_pt_theta, (size_t)(chunk + 1) * S * kThetaN)) ||
        (st = track(p, &p->d_pt_ok, (size_t)chunk * S)))
      return st;
    p->pt_cap = chunk;
  }
  if (st) return st;
  hipError_t e = stage_selection(p, m, true, sm);   // the selection, staged as the step class
  if (e == hipSuccess) e = launch_point_theta(z_fixed, S, p->d_pt_theta, nullptr, sm);
  if (e == hipSuccess) e = prep_base(p, p->d_pt_theta, sm, fp64);
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

hipError_t point_loglik(cel_plan* p, int n_cand, const double* z_cand, double* ll, hipStream_t sm,
                        const uint8_t* act, bool mark_support) {
  const bool fp64 = p->opt.pixel_fp64 != 0;
  const int S = p->S;
  const int chunk = p->pt_cap;
  const int cls = p->n_colours;
  double* th_cand = p->d_pt_theta + (int64_t)S * kThetaN;
  const int64_t row = (int64_t)S * kThetaN;
  hipError_t e = hipSuccess;
  for (int c0 = 0; c0 < n_cand && e == hipSuccess; c0 += chunk) {
    const int nc = std::min(chunk, n_cand - c0);
    e = launch_point_theta(z_cand + (int64_t)c0 * S * CEL_Z_N, (int64_t)nc * S, th_cand, p->d_pt_ok, sm);
    if (e != hipSuccess) break;
    double* out = ll + (int64_t)c0 * S;
    const uint8_t* act_c = act ? act + (int64_t)c0 * S : nullptr;
    e = fp64 ? enqueue_eval<double>(p, th_cand, nullptr, 0, nc, false, cls, nullptr, sm, false, out, nullptr, row, act_c)
             : enqueue_eval<float>(p, th_cand, nullptr, 0, nc, false, cls, nullptr, sm, false, out, nullptr, row, act_c);
    if (e == hipSuccess && mark_support) e = launch_support_masked(p->d_pt_ok, p->d_mask, S, (int64_t)nc * S, out, sm);
  }
  return e;
}

}  // namespace celmi

extern "C" cel_status cel_loglik(cel_ctx* ctx, const cel_plan* cplan, const double* z_fixed, int32_t n_cand,
                                 const double* z_cand, const uint8_t* mask, double* ll, void* stream) {
  if (!ctx || !cplan || n_cand < 0) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (p->S > 0 && n_cand > 0 && (!z_fixed || !z_cand || !ll)) return CEL_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  if (p->S == 0 || n_cand == 0) return CEL_OK;
  hipStream_t sm = (hipStream_t)stream;
  const int S = p->S;
  std::vector<uint8_t> m(S, 1);
  if (mask)
    for (int s = 0; s < S; ++s) m[s] = mask[s] ? 1 : 0;
  bool any = false;
  for (int s = 0; s < S; ++s) any = any || m[s];
  if (!any) return CEL_OK;
  cel_status st = point_setup(p, z_fixed, m, std::min<int>(n_cand, kVariants), sm);
  if (st) return st;
  return point_loglik(p, n_cand, z_cand, ll, sm) == hipSuccess ? CEL_OK : CEL_EHIP;
}

extern "C" cel_status cel_log_prior(cel_ctx* ctx, const cel_plan* plan, int64_t n, const double* z, double* out,
                                    void* stream) {
  if (!ctx || !plan || n < 0 || (n > 0 && (!z || !out))) return CEL_EINVAL;
  if (n == 0) return CEL_OK;
  if (hipSetDevice(plan->device) != hipSuccess) return CEL_EHIP;
  return launch_log_prior(plan->d_prior, z, n, out, (hipStream_t)stream) == hipSuccess ? CEL_OK : CEL_EHIP;
}

static bool valid_chunk(int c) { return c >= 64 && c % 64 == 0 && c <= (1 << 20); }
static bool valid_ppl(int c) { return c == 1 || c == 2 || c == 4; }
static bool valid_map(int c) { return c == -1 || c == 1 || c == 2 || c == 4 || c == 8; }

extern "C" cel_status cel_tune(cel_ctx* ctx, cel_plan* p, const double* theta, const cel_tune_space* space,
                               cel_tuning* out, void* stream) {
  if (!ctx || !p || (!theta && p->S > 0)) return CEL_EINVAL;
  std::vector<int> chunks{256, 512, 1024, 2048}, ppls{1, 2, 4}, maps{1, 2, 4, 8, -1};
  if (space) {
    if (space->n_chunk < 0 || space->n_chunk > 8 || space->n_pixels_per_lane < 0 || space->n_pixels_per_lane > 4 ||
        space->n_map < 0 || space->n_map > 6)
      return CEL_EINVAL;
    chunks.assign(space->chunk_pixels, space->chunk_pixels + space->n_chunk);
    ppls.assign(space->pixels_per_lane, space->pixels_per_lane + space->n_pixels_per_lane);
    maps.assign(space->map_pixels_per_lane, space->map_pixels_per_lane + space->n_map);
  }
  for (int c : chunks)
    if (!valid_chunk(c)) return CEL_EINVAL;
  for (int c : ppls)
    if (!valid_ppl(c)) return CEL_EINVAL;
  for (int c : maps)
    if (!valid_map(c)) return CEL_EINVAL;
  if (chunks.empty()) chunks.push_back(p->opt.chunk_pixels);
  if (ppls.empty()) ppls.push_back(p->opt.pixels_per_lane);
  if (maps.empty()) maps.push_back(p->opt.map_pixels_per_lane);
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  cel_tuning res{p->opt.chunk_pixels, p->opt.pixels_per_lane, p->opt.map_pixels_per_lane, 0, 0.0};
  if (p->S == 0) {
    if (out) *out = res;
    return CEL_OK;
  }
  hipStream_t sm = (hipStream_t)stream;
  const bool fp64 = p->opt.pixel_fp64 != 0;
  constexpr int kReps = 5;
  hipEvent_t ev[kReps + 1] = {};
  for (auto& x : ev)
    if (hipEventCreate(&x) != hipSuccess) {
      for (auto& y : ev)
        if (y) (void)hipEventDestroy(y);
      return CEL_EHIP;
    }
  const bool marking = p->marking;
  p->marking = false;
  // the least time of kReps evaluations after a warm-up, in ms (negative on a HIP error)
  auto time_it = [&]() -> double {
    hipError_t e = eval_any(p, theta, nullptr, 0, 1, true, -1, nullptr, sm, true, fp64);
    for (int r = 0; r <= kReps && e == hipSuccess; ++r) {
      e = hipEventRecord(ev[r], sm);
      if (e == hipSuccess && r < kReps) e = eval_any(p, theta, nullptr, 0, 1, true, -1, nullptr, sm, true, fp64);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[kReps]);
    double best = INFINITY;
    for (int r = 0; r < kReps && e == hipSuccess; ++r) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
      best = std::min(best, (double)ms);
    }
    ++res.n_timed;
    return e == hipSuccess ? best : -1.0;
  };
  // a candidate replaces the kept setting only when it is faster by more than the margin:
  // settings within a few percent of each other trade places from run to run, and a choice
  // that flips would change the plan's results in their last bits
  constexpr double kMargin = 0.05;
  constexpr int kPasses = 2, kWarm = 40;
  const int cur_chunk = p->opt.chunk_pixels, cur_ppl = p->opt.pixels_per_lane, cur_map = p->opt.map_pixels_per_lane;
  cel_status st = CEL_OK;
  // the device's clocks settle before anything is timed: evaluations right after an idle
  // spell run slower while the clocks ramp, which would count against whatever came first
  {
    hipError_t e = hipSuccess;
    for (int r = 0; r < kWarm && e == hipSuccess; ++r) e = eval_any(p, theta, nullptr, 0, 1, true, -1, nullptr, sm, true, fp64);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) st = CEL_EHIP;
  }
  // each candidate's time: the least over kPasses passes through all candidates (a drift of
  // the clocks during the search then favours none of them); the fastest replaces the
  // plan's setting when it beats it by the margin (or the setting is not a candidate)
  auto pick = [&](const std::vector<double>& t, int cur) {
    int f = 0;
    for (int i = 1; i < (int)t.size(); ++i)
      if (t[i] < t[f]) f = i;
    return (cur >= 0 && !(t[f] < t[cur] * (1.0 - kMargin))) ? cur : f;
  };
  // work-item size and pixel-pass lanes together (the pass's cost depends on both) ...
  const int np = (int)ppls.size();
  std::vector<double> t_pair(chunks.size() * np, INFINITY);
  for (int pass = 0; pass < kPasses && !st; ++pass)
    for (int ci = 0; ci < (int)chunks.size() && !st; ++ci) {
      if ((st = plan_retile(p, chunks[ci], sm)) || (st = ensure_variants(p, 1, fp64))) break;
      for (int li = 0; li < np; ++li) {
        p->opt.pixels_per_lane = ppls[li];
        const double ms = time_it();
        if (ms < 0) {
          st = CEL_EHIP;
          break;
        }
        t_pair[ci * np + li] = std::min(t_pair[ci * np + li], ms);
      }
    }
  double best_ms = INFINITY;
  if (!st) {
    int cur = -1;
    for (int i = 0; i < (int)t_pair.size(); ++i)
      if (chunks[i / np] == cur_chunk && ppls[i % np] == cur_ppl) cur = i;
    const int k = pick(t_pair, cur);
    res.chunk_pixels = chunks[k / np];
    res.pixels_per_lane = ppls[k % np];
    best_ms = t_pair[k];
    st = plan_retile(p, res.chunk_pixels, sm);
  }
  if (!st) st = ensure_variants(p, 1, fp64);
  // ... then the moment-map variants at the chosen pair
  if (!st) {
    p->opt.pixels_per_lane = res.pixels_per_lane;
    std::vector<double> t_map(maps.size(), INFINITY);
    for (int pass = 0; pass < kPasses && !st; ++pass)
      for (int mi = 0; mi < (int)maps.size(); ++mi) {
        p->opt.map_pixels_per_lane = maps[mi];
        const double ms = time_it();
        if (ms < 0) {
          st = CEL_EHIP;
          break;
        }
        t_map[mi] = std::min(t_map[mi], ms);
      }
    if (!st) {
      int cur = -1;
      for (int i = 0; i < (int)maps.size(); ++i)
        if (maps[i] == cur_map) cur = i;
      const int k = pick(t_map, cur);
      res.map_pixels_per_lane = maps[k];
      best_ms = t_map[k];
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  p->marking = marking;
  p->opt.pixels_per_lane = res.pixels_per_lane;
  p->opt.map_pixels_per_lane = res.map_pixels_per_lane;
  res.ms_per_eval = best_ms;
  // sweep graphs captured with another setting are rebuilt on their next use
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
  if (out) *out = res;
  return st;
}

extern "C" cel_status cel_phase_times(cel_plan* p, double* ms, int64_t* n_calls, int32_t reset) {
  if (!p || !p->opt.timing) return CEL_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  double acc[4] = {0, 0, 0, 0};
  int64_t n = 0;
  for (auto& r : p->ev_rec) {
    if (hipEventSynchronize(r[4]) != hipSuccess) return CEL_EHIP;
    for (int k = 0; k < 4; ++k) {
      float t = 0;
      if (hipEventElapsedTime(&t, r[k], r[k + 1]) != hipSuccess) return CEL_EHIP;
      acc[k] += t;
    }
    ++n;
  }
  if (ms)
    for (int k = 0; k < 4; ++k) ms[k] = acc[k];
  if (n_calls) *n_calls = n;
  if (reset) {
    for (auto& r : p->ev_rec)
      for (hipEvent_t e : r) p->ev_pool.push_back(e);
    p->ev_rec.clear();
  }
  return CEL_OK;
}
