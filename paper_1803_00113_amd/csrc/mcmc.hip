// MCMC source step (gfx950): annealed importance sampling over temperatures with
// slice-sampling-within-Gibbs transitions, then further slice-sampling chains at the target
// and Bayes' rule over the source type (Section 3, equation eqzs; Section 3.1: the type's
// marginal likelihood by annealed importance sampling from the prior; Section 3.2: the
// chains that follow and the draw of the type and of one sample).
//
// Every chain (source s, type a, run r) is a small state machine in device memory.  The
// chains of all selected sources advance in lockstep rounds: each round every chain asks for
// the log target at one candidate point, all candidates are evaluated in one batched
// likelihood pass (one variant of the pixel pass per candidate, the neighbours at z_fixed)
// plus the prior density, and k_mcmc_advance consumes the values and emits each chain's next
// candidate.  Chains need different numbers of evaluations (stepping out and shrinkage are
// data dependent), so they drift apart in (temperature, coordinate); a finished chain
// re-submits its point until every chain is done.
//
// The univariate update is Neal's slice sampler with stepping out and shrinkage; random
// numbers come from Philox4x64-10 (Salmon et al., SC 2011) at counters fixed by (chain,
// sweep, coordinate, draw), so the sequence of each chain does not depend on the rounds.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace celmi {

// runs per source type: both types' chains of a source are candidates of one likelihood
// launch, at most kVariants of them
constexpr int kMcmcMaxRuns = kVariants / 2;

enum McmcPhase : int32_t { PH_INIT = 0, PH_STEP_L = 1, PH_STEP_R = 2, PH_SHRINK = 3, PH_DONE = 4 };

struct McmcChain {
  double z[CEL_Z_N];      // current point
  double lp, ll;          // log prior and log likelihood at z
  double logw;            // annealed importance sampling log weight
  double y, L, R, x1;     // current slice update: threshold, interval, candidate
  int32_t t;              // sweep: 1..T annealing, T+1..T+B' at the target
  int32_t ci;             // index into the type's coordinate list
  int32_t phase, J, K, shrink;
  int32_t n_eval;         // candidates evaluated (statistics)
  int32_t pad;
};

struct McmcArgs {
  int32_t S, n_sel, n_runs, n_post, n_temps, max_step_out, max_shrink;
  const int32_t* sel;         // [n_sel] selected sources
  McmcChain* chains;          // [n_sel][2 n_runs]
  const double* z_fixed;      // [S][16]
  const double* z_init;       // [2][n_runs][S][16]
  double* z_cand;             // [2 n_runs][S][16]
  const double* ll_cand;      // [2 n_runs][S]
  const double* lp_cand;      // [2 n_runs][S]
  double* samples;            // [S][2][n_runs][n_post][16]
  const double* gamma;        // [T + 1]
  double width[CEL_Z_N];
  double box;
  uint64_t key0, key1;
  uint8_t* act;               // [2 n_runs][S]: the chain of (candidate, source) still runs
};

// ---------------------------------------------------------------------------------------
// Philox4x64-10

struct U4 {
  uint64_t v[4];
};

__device__ __forceinline__ U4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  U4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// a 64-bit word as a uniform in (0, 1): ((x >> 11) + 1/2) 2^-53
__device__ __forceinline__ double to_uniform(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

// the coordinates of the point a sweep updates, per type (1 star, 0 galaxy)
__constant__ int32_t c_coords[2][11] = {{0, 1, 3, 4, 5, 6, 7, 8, 9, 10, 11}, {0, 1, 3, 4, 5, 6, 7, 0, 0, 0, 0}};
__constant__ int32_t c_ncoords[2] = {11, 7};
constexpr int kAngle = 8;

__device__ __forceinline__ double combine(double lp, double ll, double g) {
  return (lp == -INFINITY || ll == -INFINITY) ? -INFINITY : lp + g * ll;
}

// The chain's temperature factor in its current sweep.
__device__ __forceinline__ double chain_gamma(const McmcArgs& a, int t) { return t <= a.n_temps ? a.gamma[t] : 1.0; }

// Start the slice update of coordinate ci in sweep t; returns the first candidate value.
__device__ double begin_update(const McmcArgs& a, McmcChain& c, int type, uint64_t chain_id) {
  const int coord = c_coords[type][c.ci];
  const double x0 = c.z[coord], w = a.width[coord];
  const U4 d = philox4x64(0, (uint64_t)(16 * c.t + c.ci), chain_id, 0, a.key0, a.key1);
  c.y = combine(c.lp, c.ll, chain_gamma(a, c.t)) + log(to_uniform(d.v[0]));
  c.L = x0 - w * to_uniform(d.v[1]);
  c.R = c.L + w;
  c.J = (int)floor(a.max_step_out * to_uniform(d.v[2]));
  c.K = (a.max_step_out - 1) - c.J;
  c.shrink = 0;
  if (c.J > 0) {
    c.phase = PH_STEP_L;
    return c.L;
  }
  if (c.K > 0) {
    c.phase = PH_STEP_R;
    return c.R;
  }
  c.phase = PH_SHRINK;
  const U4 u = philox4x64(1, (uint64_t)(16 * c.t + c.ci), chain_id, 0, a.key0, a.key1);
  c.x1 = c.L + to_uniform(u.v[0]) * (c.R - c.L);
  return c.x1;
}

__device__ __forceinline__ double shrink_candidate(const McmcArgs& a, McmcChain& c, uint64_t chain_id) {
  const U4 u = philox4x64(1 + (uint64_t)c.shrink, (uint64_t)(16 * c.t + c.ci), chain_id, 0, a.key0, a.key1);
  c.x1 = c.L + to_uniform(u.v[0]) * (c.R - c.L);
  c.phase = PH_SHRINK;
  return c.x1;
}

// After a coordinate's update: the next coordinate, sweep, annealing weight and sample.
// Returns the next candidate value (or NAN when the chain is done).
__device__ double next_coordinate(const McmcArgs& a, McmcChain& c, int type, uint64_t chain_id, double* smp) {
  c.ci += 1;
  if (c.ci == c_ncoords[type]) {
    if (c.t > a.n_temps) {
      double* o = smp + (int64_t)(c.t - a.n_temps - 1) * CEL_Z_N;
#pragma unroll
      for (int k = 0; k < CEL_Z_N; ++k) o[k] = c.z[k];
    }
    c.ci = 0;
    c.t += 1;
    if (c.t > a.n_temps + a.n_post) {
      c.phase = PH_DONE;
      return NAN;
    }
    if (c.t <= a.n_temps) c.logw += (a.gamma[c.t] - a.gamma[c.t - 1]) * c.ll;
  }
  return begin_update(a, c, type, chain_id);
}

// One thread per chain: consume the evaluated candidate, emit the next one.
__global__ __launch_bounds__(256) void k_mcmc_advance(McmcArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nch = 2 * a.n_runs;
  if (i >= a.n_sel * nch) return;
  const int js = i / nch, cc = i - js * nch;           // selected source, chain within it
  const int s = a.sel[js];
  const int type = cc >= a.n_runs ? 1 : 0, run = cc - type * a.n_runs;
  const uint64_t chain_id = (uint64_t)(2 * s + type) * (uint64_t)a.n_runs + (uint64_t)run;
  McmcChain c = a.chains[i];
  double* smp = a.samples + (((int64_t)s * 2 + type) * a.n_runs + run) * (int64_t)a.n_post * CEL_Z_N;
  double* cand = a.z_cand + ((int64_t)cc * a.S + s) * CEL_Z_N;
  if (c.phase == PH_DONE) return;   // its candidate row still holds its point, not evaluated
  // the evaluated candidate: log prior, log likelihood, the position's box
  const int64_t at = (int64_t)cc * a.S + s;
  double lpc = a.lp_cand[at], llc = a.ll_cand[at];
  if (fabs(cand[0] - a.z_fixed[(int64_t)s * CEL_Z_N]) > a.box || fabs(cand[1] - a.z_fixed[(int64_t)s * CEL_Z_N + 1]) > a.box ||
      lpc == -INFINITY) {
    lpc = -INFINITY;
    llc = -INFINITY;
  }
  c.n_eval += 1;
  double next = NAN;
  if (c.phase == PH_INIT) {
    c.lp = lpc;
    c.ll = llc;
    c.t = 1;
    c.ci = 0;
    c.logw = (a.gamma[1] - a.gamma[0]) * c.ll;
    next = begin_update(a, c, type, chain_id);
  } else {
    const int coord = c_coords[type][c.ci];
    const double w = a.width[coord];
    const double f = combine(lpc, llc, chain_gamma(a, c.t));
    if (c.phase == PH_STEP_L) {
      bool more = false;
      if (c.y < f) {
        c.L -= w;
        c.J -= 1;
        more = c.J > 0;
      }
      if (more) {
        next = c.L;
      } else if (c.K > 0) {
        c.phase = PH_STEP_R;
        next = c.R;
      } else {
        next = shrink_candidate(a, c, chain_id);
      }
    } else if (c.phase == PH_STEP_R) {
      bool more = false;
      if (c.y < f) {
        c.R += w;
        c.K -= 1;
        more = c.K > 0;
      }
      next = more ? c.R : shrink_candidate(a, c, chain_id);
    } else {   // PH_SHRINK
      const double x0 = c.z[coord];
      if (c.y < f) {
        double x1 = c.x1;
        if (coord == kAngle) x1 = x1 - M_PI * floor(x1 / M_PI);   // period pi
        c.z[coord] = x1;
        c.lp = lpc;
        c.ll = llc;
        next = next_coordinate(a, c, type, chain_id, smp);
      } else {
        if (c.x1 < x0)
          c.L = c.x1;
        else
          c.R = c.x1;
        c.shrink += 1;
        next = c.shrink >= a.max_shrink ? next_coordinate(a, c, type, chain_id, smp)
                                        : shrink_candidate(a, c, chain_id);
      }
    }
  }
  // the next candidate: the point with the coordinate being updated replaced
#pragma unroll
  for (int k = 0; k < CEL_Z_N; ++k) cand[k] = c.z[k];
  if (c.phase != PH_DONE) cand[c_coords[type][c.ci]] = next;
  a.chains[i] = c;
  // a finished chain's candidate is not evaluated again
  if (c.phase == PH_DONE) a.act[at] = 0;
}

// Chains from their start points; every candidate row of a selected source its start point.
__global__ __launch_bounds__(256) void k_mcmc_init(McmcArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nch = 2 * a.n_runs;
  if (i >= a.n_sel * nch) return;
  const int js = i / nch, cc = i - js * nch;
  const int s = a.sel[js];
  const int type = cc >= a.n_runs ? 1 : 0, run = cc - type * a.n_runs;
  McmcChain c;
  const double* z0 = a.z_init + (((int64_t)type * a.n_runs + run) * a.S + s) * CEL_Z_N;
  double* cand = a.z_cand + ((int64_t)cc * a.S + s) * CEL_Z_N;
#pragma unroll
  for (int k = 0; k < CEL_Z_N; ++k) {
    c.z[k] = z0[k];
  }
  c.z[2] = (double)type;
#pragma unroll
  for (int k = 0; k < CEL_Z_N; ++k) cand[k] = c.z[k];
  c.lp = c.ll = c.logw = c.y = c.L = c.R = c.x1 = 0.0;
  c.t = c.ci = c.J = c.K = c.shrink = c.n_eval = c.pad = 0;
  c.phase = PH_INIT;
  a.chains[i] = c;
  a.act[(int64_t)cc * a.S + s] = 1;
}

// Rows of unselected sources: their fixed point (the likelihood pass reads every row).
__global__ __launch_bounds__(256) void k_mcmc_fill(const double* z_fixed, const uint8_t* sel_mask, int S, int n_cand,
                                                   double* z_cand) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_cand * S) return;
  const int s = (int)(i % S);
  if (sel_mask[s]) return;
#pragma unroll
  for (int k = 0; k < CEL_Z_N; ++k) z_cand[i * CEL_Z_N + k] = z_fixed[(int64_t)s * CEL_Z_N + k];
}

// Chains not yet done (one workgroup; fixed-order sum).
__global__ __launch_bounds__(256) void k_mcmc_active(const McmcChain* chains, int n, int32_t* out) {
  __shared__ int32_t sh[256];
  int32_t v = 0;
  for (int i = threadIdx.x; i < n; i += 256) v += chains[i].phase != PH_DONE ? 1 : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Per selected source: evidence of each type from its runs' weights, p(a = 1 | x, z_-s) by
// Bayes' rule with the prior probability of a star, the type drawn from it and one of that
// type's samples drawn uniformly.
__global__ __launch_bounds__(64) void k_mcmc_finish(McmcArgs a, double log_odds_prior, double* z_out, double* p_star,
                                                    double* log_ev, int64_t* n_eval) {
  const int js = blockIdx.x * blockDim.x + threadIdx.x;
  if (js >= a.n_sel) return;
  const int s = a.sel[js];
  const int nch = 2 * a.n_runs;
  double ev[2];
  int64_t ne = 0;
  for (int type = 0; type < 2; ++type) {
    double mx = -INFINITY;
    for (int r = 0; r < a.n_runs; ++r) mx = fmax(mx, a.chains[(int64_t)js * nch + type * a.n_runs + r].logw);
    double sum = 0.0;
    for (int r = 0; r < a.n_runs; ++r) sum += exp(a.chains[(int64_t)js * nch + type * a.n_runs + r].logw - mx);
    ev[type] = isfinite(mx) ? mx + log(sum) - log((double)a.n_runs) : -INFINITY;
    for (int r = 0; r < a.n_runs; ++r) ne += a.chains[(int64_t)js * nch + type * a.n_runs + r].n_eval;
  }
  const double d = log_odds_prior + ev[1] - ev[0];
  const double p = d > -700.0 ? 1.0 / (1.0 + exp(-d)) : 0.0;
  const U4 u = philox4x64(0, 0, (uint64_t)s, 1, a.key0, a.key1);
  const int type = to_uniform(u.v[0]) < p ? 1 : 0;
  const int nb = a.n_runs * a.n_post;
  const int j = min((int)floor(to_uniform(u.v[1]) * nb), nb - 1);
  const double* smp = a.samples + ((((int64_t)s * 2 + type) * a.n_runs + j / a.n_post) * a.n_post + j % a.n_post) * CEL_Z_N;
  for (int k = 0; k < CEL_Z_N; ++k) z_out[(int64_t)s * CEL_Z_N + k] = smp[k];
  p_star[s] = p;
  log_ev[2 * s] = ev[0];
  log_ev[2 * s + 1] = ev[1];
  if (n_eval) n_eval[s] = ne;
}

// Potential scale reduction factor (Gelman and Rubin 1992) of each selected source's n_runs
// chains of n_post draws, per type and coordinate: the criterion with which the chains of
// Section 3.2 are monitored.  B = n / (m - 1) sum_j (mean_j - g)^2, W = mean_j s_j^2 (chain
// variances with divisor n - 1), V = (n - 1) / n W + B / n, R = sqrt(V / W) (0 / 0 = NaN for
// a coordinate no chain moves).  One thread per (selected source, type, coordinate), FP64,
// sums in chain and draw order.
__global__ __launch_bounds__(256) void k_mcmc_rhat(McmcArgs a, double* rhat) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)a.n_sel * 2 * CEL_Z_N) return;
  const int k = (int)(id % CEL_Z_N), type = (int)((id / CEL_Z_N) % 2), js = (int)(id / (2 * CEL_Z_N));
  const int s = a.sel[js];
  const int m = a.n_runs, n = a.n_post;
  double* out = rhat + ((int64_t)s * 2 + type) * CEL_Z_N + k;
  if (m < 2 || n < 2) {
    *out = NAN;
    return;
  }
  const double* x = a.samples + ((int64_t)s * 2 + type) * m * (int64_t)n * CEL_Z_N + k;
  double mean[kMcmcMaxRuns];
  double g = 0.0;
  for (int j = 0; j < m; ++j) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += x[((int64_t)j * n + i) * CEL_Z_N];
    mean[j] = t / n;
    g += mean[j];
  }
  g /= m;
  double b = 0.0, w = 0.0;
  for (int j = 0; j < m; ++j) {
    const double d = mean[j] - g;
    b += d * d;
    double v = 0.0;
    for (int i = 0; i < n; ++i) {
      const double e = x[((int64_t)j * n + i) * CEL_Z_N] - mean[j];
      v += e * e;
    }
    w += v / (n - 1);
  }
  const double B = (double)n / (m - 1) * b, W = w / m;
  const double V = (double)(n - 1) / n * W + B / n;
  *out = sqrt(V / W);
}

}  // namespace celmi

using namespace celmi;

namespace {
// a grow-only device block owned by the plan (freed with it)
template <typename X>
cel_status grow(cel_plan* p, X** ptr, size_t* cap, size_t n) {
  if (*cap >= n && *ptr) return CEL_OK;
  void* q = nullptr;
  size_t got = 0;
  cel_status st = ctx_alloc(p->ctx, std::max<size_t>(n, 1) * sizeof(X), &q, &got);
  if (st) return st;
  p->allocs.push_back({q, got});
  *ptr = static_cast<X*>(q);
  *cap = n;
  return CEL_OK;
}
}  // namespace

extern "C" cel_status cel_mcmc_step(cel_ctx* ctx, const cel_plan* cplan, const double* z_fixed, const uint8_t* mask,
                                    const double* z_init, const cel_mcmc_opts* opts, uint64_t key, double* z_out,
                                    double* p_star, double* log_evidence, double* samples, double* rhat,
                                    cel_mcmc_report* report, void* stream) {
  if (!ctx || !cplan || !opts) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  const cel_mcmc_opts& o = *opts;
  if (o.n_temps < 1 || o.n_runs < 1 || o.n_post < 1 || o.max_step_out < 1 || o.max_shrink < 1 || !o.gamma ||
      !(o.box > 0) || o.n_runs > kMcmcMaxRuns)
    return CEL_EINVAL;
  if (o.n_temps > (1 << 24) || o.n_post > (1 << 20)) return CEL_EUNSUPPORTED;
  for (int k = 0; k < CEL_Z_N; ++k)
    if (!(o.width[k] >= 0) || !std::isfinite(o.width[k])) return CEL_EINVAL;
  const int S = p->S;
  if (S > 0 && (!z_fixed || !z_init || !z_out || !p_star || !log_evidence)) return CEL_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  std::vector<uint8_t> m(S, 1);
  if (mask)
    for (int s = 0; s < S; ++s) m[s] = mask[s] ? 1 : 0;
  std::vector<int32_t> sel;
  for (int s = 0; s < S; ++s)
    if (m[s]) sel.push_back(s);
  if (report) std::memset(report, 0, sizeof(*report));
  if (sel.empty()) return CEL_OK;
  hipStream_t sm = (hipStream_t)stream;
  const int n_sel = (int)sel.size(), nch = 2 * o.n_runs, n_chains = n_sel * nch;
  cel_status st = point_setup(p, z_fixed, m, nch, sm);
  if (st) return st;
  // the sampler's scratch: chains, candidate rows and their values, samples, the selection
  static_assert(sizeof(McmcChain) % 8 == 0, "chain records are float64-aligned");
  const size_t n_smp = (size_t)S * 2 * o.n_runs * o.n_post * CEL_Z_N;
  if ((st = grow(p, &p->mc_chains, &p->mc_chains_cap, (size_t)n_chains * sizeof(McmcChain))) ||
      (st = grow(p, &p->mc_cand, &p->mc_cand_cap, (size_t)nch * S * CEL_Z_N)) ||
      (st = grow(p, &p->mc_vals, &p->mc_vals_cap, (size_t)2 * nch * S)) ||
      (st = grow(p, &p->mc_act, &p->mc_act_cap, (size_t)nch * S)) ||
      (st = grow(p, &p->mc_sel, &p->mc_sel_cap, (size_t)n_sel + S + 2)) ||
      (!samples && (st = grow(p, &p->mc_samples, &p->mc_samples_cap, n_smp))))
    return st;
  int32_t* d_sel = p->mc_sel;
  uint8_t* d_selmask = reinterpret_cast<uint8_t*>(p->mc_sel + n_sel);
  int32_t* d_active = p->mc_sel + n_sel + (S + 3) / 4 + 1;
  std::vector<int32_t> up(n_sel + (S + 3) / 4 + 1, 0);
  std::memcpy(up.data(), sel.data(), sizeof(int32_t) * n_sel);
  std::memcpy(reinterpret_cast<char*>(up.data() + n_sel), m.data(), S);
  if ((st = grow(p, &p->mc_gamma, &p->mc_gamma_cap, (size_t)o.n_temps + 1))) return st;
  double* d_gamma = p->mc_gamma;
  hipError_t e = hipMemcpyAsync(d_sel, up.data(), sizeof(int32_t) * up.size(), hipMemcpyHostToDevice, sm);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_gamma, o.gamma, sizeof(double) * (o.n_temps + 1), hipMemcpyHostToDevice, sm);
  // (the host vectors must outlive the copies)
  if (e == hipSuccess) e = hipStreamSynchronize(sm);
  if (e != hipSuccess) return CEL_EHIP;
  McmcArgs a;
  std::memset(&a, 0, sizeof(a));
  a.S = S;
  a.n_sel = n_sel;
  a.n_runs = o.n_runs;
  a.n_post = o.n_post;
  a.n_temps = o.n_temps;
  a.max_step_out = o.max_step_out;
  a.max_shrink = o.max_shrink;
  a.sel = d_sel;
  a.chains = reinterpret_cast<McmcChain*>(p->mc_chains);
  a.z_fixed = z_fixed;
  a.z_init = z_init;
  a.z_cand = p->mc_cand;
  a.act = p->mc_act;
  a.ll_cand = p->mc_vals;
  a.lp_cand = p->mc_vals + (size_t)nch * S;
  a.samples = samples ? samples : p->mc_samples;
  a.gamma = d_gamma;
  for (int k = 0; k < CEL_Z_N; ++k) a.width[k] = o.width[k];
  a.box = o.box;
  a.key0 = o.seed;
  a.key1 = key;
  double* ll_c = p->mc_vals;
  double* lp_c = p->mc_vals + (size_t)nch * S;
  const int blocks = (n_chains + 255) / 256;
  const int64_t rows = (int64_t)nch * S;
  hipLaunchKernelGGL(k_mcmc_fill, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, sm, z_fixed, d_selmask, S, nch,
                     p->mc_cand);
  hipLaunchKernelGGL(k_mcmc_init, dim3(blocks), dim3(256), 0, sm, a);
  e = hipGetLastError();
  int64_t rounds = 0;
  const int kCheck = 16;
  int32_t* h_active = p->h_counter;   // pinned word of the plan's Newton kit
  while (e == hipSuccess) {
    for (int r = 0; r < kCheck && e == hipSuccess; ++r, ++rounds) {
      // (a candidate outside the support has log prior -infinity, which the advance reads
      // as a rejected point: the likelihood pass need not mark it)
      e = point_loglik(p, nch, p->mc_cand, ll_c, sm, p->mc_act, false);
      if (e == hipSuccess) e = launch_log_prior(p->d_prior, p->mc_cand, rows, lp_c, sm);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mcmc_advance, dim3(blocks), dim3(256), 0, sm, a);
        e = hipGetLastError();
      }
    }
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_mcmc_active, dim3(1), dim3(256), 0, sm, (const McmcChain*)a.chains, n_chains, d_active);
    e = hipMemcpyAsync(h_active, d_active, sizeof(int32_t), hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess || *h_active == 0) break;
  }
  if (e == hipSuccess) {
    int64_t* d_ne = reinterpret_cast<int64_t*>(p->mc_vals);   // reused: the values are no longer needed
    hipLaunchKernelGGL(k_mcmc_finish, dim3((n_sel + 63) / 64), dim3(64), 0, sm, a, p->prior_h.log_a - p->prior_h.log_1ma, z_out,
                       p_star, log_evidence, report ? d_ne : (int64_t*)nullptr);
    e = hipGetLastError();
    if (e == hipSuccess && rhat) {
      const int64_t n_r = (int64_t)n_sel * 2 * CEL_Z_N;
      hipLaunchKernelGGL(k_mcmc_rhat, dim3((unsigned)((n_r + 255) / 256)), dim3(256), 0, sm, a, rhat);
      e = hipGetLastError();
    }
    if (e == hipSuccess && report) {
      std::vector<int64_t> ne(S, 0);
      e = hipMemcpyAsync(ne.data(), d_ne, sizeof(int64_t) * S, hipMemcpyDeviceToHost, sm);
      if (e == hipSuccess) e = hipStreamSynchronize(sm);
      int64_t tot = 0, px = 0;
      for (int js = 0; js < n_sel; ++js) {
        const int s = sel[js];
        tot += ne[s];
        int64_t pxs = 0;
        for (int q = p->patch_ptr_h[s]; q < p->patch_ptr_h[s + 1]; ++q)
          pxs += (int64_t)p->patches_h[q].w * p->patches_h[q].h;
        px += ne[s] * pxs;
      }
      report->rounds = rounds;
      report->n_chains = n_chains;
      report->evaluations = tot;
      report->candidate_pixels = px;
    }
  }
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}
