// Trust-region Newton block step and block coordinate ascent (Sections 4.3-4.4).
//
// One Newton iteration on a set of pairwise non-overlapping sources (a colour class):
//   1. component tables of every source at the current iterate (variant 0), and of each
//      stepped source at theta +/- h e_k for the 27 parameters (variants 1..54)
//   2. the fused pixel kernel and finalisation for those 55 variants: L_s and gradients
//   3. k_trsolve, one wavefront per source: the Hessian -- its pixel part by central
//      differences of the pixel gradient (symmetrised), its KL part analytically, since the
//      tight colour-prior mixture makes the KL's higher derivatives far too large for
//      differencing -- convergence tests, eigen-decomposition of -H by cyclic
//      Jacobi in LDS (FP64), the trust-region subproblem (boundary multiplier by
//      bisection on |p(lambda)| = radius, hard case along the lowest eigenvector), and
//      the trial point
//   4. the objective at the trial points (variant 55)
//   5. k_accept: ratio of actual to predicted gain, acceptance and radius update
// Trust-region constants (the paper prints none): accept if rho > eta (0.1); radius
// shrinks to |p|/4 if rho < 1/4 and doubles (to at most radius_max) if rho > 3/4 with the
// step on the boundary; converged if |g|_inf <= gtol max(1, |L_s|/n_pix), the predicted
// gain <= ftol max(1, |L_s|), or radius < radius_min.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace celmi {

constexpr int kN = kParamN;   // 27
constexpr int kLd = kN + 1;   // padded LDS row


__device__ __forceinline__ double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

// Hessian of KL_s in the unconstrained coordinates (the same KL as the objective: the type
// KL, the normal KL of log r, the colour bound -log sum_j w_j exp(-D_j), and minus the log
// prior densities of the radius, profile and axis point masses), added into B (27 x kLd).
// KL = KL_a(eta) + KL_radius + KL_profile + KL_axis + (1 - a) K_0 + a K_1.
__device__ void kl_hessian_add(const DPrior& pr, const double* th, double B[kN][kLd]) {
  const double eta = th[2], a = sigm(eta);
  const double aa = a * (1.0 - a);
  double K[2], dK[2][kN];
  for (int i = 0; i < 2; ++i) {
    for (int k = 0; k < kN; ++k) dK[i][k] = 0.0;
    const double rm = th[3 + i], lrv = th[5 + i], rv = exp(lrv);
    const double R1 = pr.r[i][0], R2 = pr.r[i][1];
    const double q = i == 0 ? 1.0 - a : a;
    K[i] = 0.5 * (log(R2) - lrv) + (rv + (rm - R1) * (rm - R1)) / (2.0 * R2) - 0.5;
    dK[i][3 + i] = (rm - R1) / R2;
    dK[i][5 + i] = -0.5 + rv / (2.0 * R2);
    B[3 + i][3 + i] += q / R2;
    B[5 + i][5 + i] += q * rv / (2.0 * R2);
    // colour bound
    double cm[4], cv[4], lcv = 0;
    for (int k = 0; k < 4; ++k) {
      cm[k] = th[7 + 4 * i + k];
      cv[k] = exp(th[15 + 4 * i + k]);
      lcv += th[15 + 4 * i + k];
    }
    double D[CEL_N_COLOUR_COMPONENTS], mx = -1e300;
    for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) {
      double tr = 0, maha = 0;
      for (int k = 0; k < 4; ++k) {
        tr += pr.c_prec[i][j][k][k] * cv[k];
        double row = 0;
        for (int l = 0; l < 4; ++l) row += pr.c_prec[i][j][k][l] * (pr.c_mean[i][j][l] - cm[l]);
        maha += (pr.c_mean[i][j][k] - cm[k]) * row;
      }
      D[j] = 0.5 * (tr + maha - 4.0 + pr.c_logdet[i][j] - lcv);
      mx = fmax(mx, pr.c_logw[i][j] - D[j]);
    }
    double z = 0;
    for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) z += exp(pr.c_logw[i][j] - D[j] - mx);
    K[i] += -(mx + log(z));
    // grad F = sum xi dD;  hess F = sum xi (d2D - dD dD^T) + gradF gradF^T  (8 variables)
    double gF[8] = {0, 0, 0, 0, 0, 0, 0, 0}, hF[8][8];
    for (int u = 0; u < 8; ++u)
      for (int w = 0; w < 8; ++w) hF[u][w] = 0.0;
    for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) {
      const double xi = exp(pr.c_logw[i][j] - D[j] - mx) / z;
      if (xi == 0.0) continue;
      double dD[8];
      for (int k = 0; k < 4; ++k) {
        double row = 0;
        for (int l = 0; l < 4; ++l) row += pr.c_prec[i][j][k][l] * (cm[l] - pr.c_mean[i][j][l]);
        dD[k] = row;
        dD[4 + k] = 0.5 * (pr.c_prec[i][j][k][k] * cv[k] - 1.0);
      }
      for (int u = 0; u < 8; ++u) {
        gF[u] += xi * dD[u];
        for (int w = 0; w < 8; ++w) hF[u][w] -= xi * dD[u] * dD[w];
      }
      for (int k = 0; k < 4; ++k) {
        for (int l = 0; l < 4; ++l) hF[k][l] += xi * pr.c_prec[i][j][k][l];
        hF[4 + k][4 + k] += xi * 0.5 * pr.c_prec[i][j][k][k] * cv[k];
      }
    }
    for (int u = 0; u < 8; ++u)
      for (int w = 0; w < 8; ++w) hF[u][w] += gF[u] * gF[w];
    int idx[8];
    for (int k = 0; k < 4; ++k) {
      idx[k] = 7 + 4 * i + k;
      idx[4 + k] = 15 + 4 * i + k;
    }
    for (int u = 0; u < 8; ++u) {
      dK[i][idx[u]] += gF[u];
      for (int w = 0; w < 8; ++w) B[idx[u]][idx[w]] += q * hF[u][w];
    }
  }
  // type weight: dKL/deta = a(1-a) [eta - logit A + K1 - K0]
  const double t = eta - pr.logit_a + K[1] - K[0];
  B[2][2] += aa * (1.0 - 2.0 * a) * t + aa;
  for (int k = 0; k < kN; ++k) {
    const double c = aa * (dK[1][k] - dK[0][k]);
    if (c != 0.0 && k != 2) {
      B[2][k] += c;
      B[k][2] += c;
    }
  }
  // point masses
  B[24][24] += 1.0 / pr.radius[1];
  {
    const double p = sigm(th[25]);
    B[25][25] += (pr.profile[0] + pr.profile[1] - 2.0) * p * (1.0 - p);
  }
  {
    const double p = sigm(th[26]);
    B[26][26] += (pr.axis[0] + pr.axis[1] - 2.0) * p * (1.0 - p);
  }
}

struct TrArgs {
  const int32_t* job_src;     // sources of this launch
  int32_t n_jobs;
  int32_t S;
  const uint8_t* active;
  const double* v_grad;       // [variants][S][32]
  const double* v_local;      // [variants][S]
  double fd_step;
  const double* theta;
  const double* radius;
  const double* npix;         // active pixels per source
  double gtol, ftol, radius_min;
  double* theta_trial;        // out [S][32]
  uint8_t* trial_active;      // out: 1 = trial point to evaluate
  double* pred;               // out: predicted gain
  double* pnorm;              // out: |p|
  int32_t* status;            // out: CONVERGED / NONFINITE for sources not tried
  const DPrior* prior;
};

__global__ __launch_bounds__(64) void k_trsolve(TrArgs a) {
  const int s = a.job_src ? a.job_src[blockIdx.x] : (int)blockIdx.x;
  if (a.active && !a.active[s]) {
    if (threadIdx.x == 0) a.trial_active[s] = 0;
    return;
  }
  __shared__ double B[kN][kLd];
  __shared__ double V[kN][kLd];
  __shared__ double g[kN], lam[kN], y[kN], gt[kN];
  __shared__ int ok_flag;
  __shared__ double red[64];
  const int lane = threadIdx.x;
  const int64_t vs = (int64_t)a.S * kThetaN;
  const double h2 = 2.0 * a.fd_step;
  const double L = a.v_local[s];
  for (int idx = lane; idx < kN * kN; idx += 64) {
    const int i = idx / kN, k = idx % kN;
    const double hik = (a.v_grad[(int64_t)(1 + k) * vs + (int64_t)s * kThetaN + i] -
                        a.v_grad[(int64_t)(1 + kN + k) * vs + (int64_t)s * kThetaN + i]) / h2;
    B[i][k] = -hik;
    V[i][k] = (i == k) ? 1.0 : 0.0;
  }
  if (lane < kN) g[lane] = a.v_grad[(int64_t)s * kThetaN + lane];
  __syncthreads();
  // symmetrise: each unordered pair handled by one thread
  for (int idx = lane; idx < kN * kN; idx += 64) {
    const int i = idx / kN, k = idx % kN;
    if (i < k) {
      const double v = 0.5 * (B[i][k] + B[k][i]);
      B[i][k] = v;
      B[k][i] = v;
    }
  }
  __syncthreads();
  // B = -H = -(H_pixels - H_KL): the pixel part by central differences (above), the KL part
  // analytically
  if (lane == 0) {
    double th[kN];
    for (int k = 0; k < kN; ++k) th[k] = a.theta[(int64_t)s * kThetaN + k];
    kl_hessian_add(*a.prior, th, B);
  }
  __syncthreads();
  // finiteness and the gradient test
  double gm = 0.0;
  bool fin = true;
  for (int idx = lane; idx < kN * kN; idx += 64) fin = fin && isfinite(B[idx / kN][idx % kN]);
  if (lane < kN) {
    fin = fin && isfinite(g[lane]);
    gm = fabs(g[lane]);
  }
  if (lane == 0) ok_flag = 1;
  __syncthreads();
  if (!fin) ok_flag = 0;
  red[lane] = gm;
  __syncthreads();
  if (lane == 0) {
    double m = 0;
    for (int i = 0; i < 64; ++i) m = fmax(m, red[i]);
    red[0] = m;
  }
  __syncthreads();
  const double gmax = red[0];
  const double radius = a.radius[s];
  if (!ok_flag || !isfinite(L) || !isfinite(radius)) {
    if (lane == 0) {
      a.status[s] = CEL_ST_NONFINITE;
      a.trial_active[s] = 0;
    }
    return;
  }
  if (gmax <= a.gtol * fmax(1.0, fabs(L) / fmax(a.npix[s], 1.0)) || radius < a.radius_min) {
    if (lane == 0) {
      a.status[s] = CEL_ST_CONVERGED;
      a.trial_active[s] = 0;
    }
    return;
  }
  // cyclic Jacobi: B <- J^T B J, V <- V J (Golub & Van Loan, symmetric Schur 2x2 rotations)
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = lane; idx < kN * kN; idx += 64) {
      const int i = idx / kN, k = idx % kN;
      const double v = B[i][k] * B[i][k];
      tot += v;
      if (i != k) off += v;
    }
    red[lane] = off;
    __syncthreads();
    if (lane == 0) {
      double o = 0;
      for (int i = 0; i < 64; ++i) o += red[i];
      red[0] = o;
    }
    __syncthreads();
    const double offs = red[0];
    __syncthreads();
    red[lane] = tot;
    __syncthreads();
    if (lane == 0) {
      double o = 0;
      for (int i = 0; i < 64; ++i) o += red[i];
      red[0] = o;
    }
    __syncthreads();
    const double tots = red[0];
    __syncthreads();
    if (!(offs > 1e-30 * tots) || offs == 0.0) break;
    for (int p = 0; p < kN - 1; ++p) {
      for (int q = p + 1; q < kN; ++q) {
        const double apq = B[p][q];
        if (apq == 0.0) continue;
        const double app = B[p][p], aqq = B[q][q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        double bip = 0, biq = 0;
        if (lane < kN) {
          bip = B[lane][p];
          biq = B[lane][q];
        }
        __syncthreads();
        if (lane < kN) {
          B[lane][p] = c * bip - sn * biq;
          B[lane][q] = sn * bip + c * biq;
        }
        __syncthreads();
        double bpi = 0, bqi = 0, vip = 0, viq = 0;
        if (lane < kN) {
          bpi = B[p][lane];
          bqi = B[q][lane];
          vip = V[lane][p];
          viq = V[lane][q];
        }
        __syncthreads();
        if (lane < kN) {
          B[p][lane] = c * bpi - sn * bqi;
          B[q][lane] = sn * bpi + c * bqi;
          V[lane][p] = c * vip - sn * viq;
          V[lane][q] = sn * vip + c * viq;
        }
        __syncthreads();
      }
    }
  }
  if (lane < kN) lam[lane] = B[lane][lane];
  __syncthreads();
  // gt = V^T g (stored in y temporarily)
  if (lane < kN) {
    double acc = 0;
    for (int i = 0; i < kN; ++i) acc += V[i][lane] * g[i];
    y[lane] = acc;
  }
  __syncthreads();
  if (lane < kN) gt[lane] = y[lane];
  __syncthreads();
  if (lane == 0) {
    double gnorm = 0;
    for (int i = 0; i < kN; ++i) gnorm += g[i] * g[i];
    gnorm = sqrt(gnorm);
    double lmin = lam[0];
    int imin = 0;
    for (int i = 1; i < kN; ++i)
      if (lam[i] < lmin) {
        lmin = lam[i];
        imin = i;
      }
    double lamb = -1.0;   // chosen multiplier (< 0: not yet found)
    bool hard = false;
    if (lmin > 0) {
      double nn = 0;
      for (int i = 0; i < kN; ++i) nn += (gt[i] / lam[i]) * (gt[i] / lam[i]);
      if (sqrt(nn) <= radius) lamb = 0.0;
    }
    const double lo = fmax(0.0, -lmin);
    double tau_hard = 0.0;
    if (lamb < 0) {
      bool orth = true;
      for (int i = 0; i < kN; ++i)
        if (fabs(lam[i] - lmin) <= 1e-12 * fmax(1.0, fabs(lmin)) && fabs(gt[i]) > 1e-12 * fmax(gnorm, 1e-300))
          orth = false;
      if (orth) {
        double nr = 0;
        for (int i = 0; i < kN; ++i)
          if (!(fabs(lam[i] - lmin) <= 1e-12 * fmax(1.0, fabs(lmin)))) {
            const double v = gt[i] / (lam[i] + lo);
            nr += v * v;
          }
        if (sqrt(nr) <= radius) {
          hard = true;
          lamb = lo;
          tau_hard = sqrt(fmax(radius * radius - nr, 0.0));
        }
      }
    }
    if (lamb < 0) {
      auto norm_p = [&](double l) {
        double nn = 0;
        for (int i = 0; i < kN; ++i) {
          const double v = gt[i] / (lam[i] + l);
          nn += v * v;
        }
        return sqrt(nn);
      };
      double hi = lo + gnorm / radius + 1.0;
      while (norm_p(hi) > radius) hi = lo + 2.0 * (hi - lo);
      double aa = lo, bb = hi;
      for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (aa + bb);
        if (mid == aa || mid == bb) break;
        if (norm_p(mid) > radius) aa = mid;
        else bb = mid;
      }
      lamb = bb;
    }
    // step in the eigenbasis, predicted gain and norm
    double gp = 0, pBp = 0, nn = 0;
    for (int i = 0; i < kN; ++i) {
      double yi;
      if (hard && fabs(lam[i] - lmin) <= 1e-12 * fmax(1.0, fabs(lmin))) yi = 0.0;
      else yi = gt[i] / (lam[i] + lamb);
      y[i] = yi;
    }
    if (hard) {
      // orient the lowest eigenvector so its largest-magnitude entry is positive
      int am = 0;
      for (int i = 1; i < kN; ++i)
        if (fabs(V[i][imin]) > fabs(V[am][imin])) am = i;
      y[imin] = V[am][imin] < 0 ? -tau_hard : tau_hard;
    }
    for (int i = 0; i < kN; ++i) {
      gp += gt[i] * y[i];
      pBp += lam[i] * y[i] * y[i];
      nn += y[i] * y[i];
    }
    const double pr = gp - 0.5 * pBp;
    a.pred[s] = pr;
    a.pnorm[s] = sqrt(nn);
    if (!(pr > a.ftol * fmax(1.0, fabs(L)))) {
      a.status[s] = CEL_ST_CONVERGED;
      a.trial_active[s] = 0;
      ok_flag = 0;
    } else {
      a.trial_active[s] = 1;
      ok_flag = 1;
    }
  }
  __syncthreads();
  if (!ok_flag) return;
  if (lane < kThetaN) {
    double v = a.theta[(int64_t)s * kThetaN + lane];
    if (lane < kN) {
      double step = 0;
      for (int i = 0; i < kN; ++i) step += V[lane][i] * y[i];
      v += step;
    }
    a.theta_trial[(int64_t)s * kThetaN + lane] = v;
  }
}

struct AcceptArgs {
  const int32_t* job_src;
  int32_t n_jobs;
  uint8_t* active;            // stepped sources (cleared on convergence when clear_done)
  int32_t clear_done;
  const uint8_t* trial_active;
  const double* local0;       // L_s at the iterate
  const double* local_trial;  // L_s at the trial point
  const double* pred;
  const double* pnorm;
  double* theta;
  const double* theta_trial;
  double* radius;
  int32_t* status;
  double* out_local;          // may be null
  double eta, radius_max;
};

__global__ __launch_bounds__(64) void k_accept(AcceptArgs a) {
  const int jj = blockIdx.x * 64 + threadIdx.x;
  if (jj >= a.n_jobs) return;
  const int s = a.job_src ? a.job_src[jj] : jj;
  if (!a.active[s]) return;
  const double L = a.local0[s];
  double Lout = L;
  if (a.trial_active[s]) {
    const double Lt = a.local_trial[s];
    const double pn = a.pnorm[s];
    double r = a.radius[s];
    int st;
    if (!isfinite(Lt)) {
      r = 0.25 * pn;
      st = CEL_ST_REJECTED;
    } else {
      const double rho = (Lt - L) / a.pred[s];
      if (rho < 0.25) r = 0.25 * pn;
      else if (rho > 0.75 && pn >= 0.99 * r) r = fmin(2.0 * r, a.radius_max);
      if (rho > a.eta) {
        st = CEL_ST_ACCEPTED;
        for (int k = 0; k < kThetaN; ++k) a.theta[(int64_t)s * kThetaN + k] = a.theta_trial[(int64_t)s * kThetaN + k];
        Lout = Lt;
      } else {
        st = CEL_ST_REJECTED;
      }
    }
    a.radius[s] = r;
    a.status[s] = st;
  } else if (a.clear_done) {
    a.active[s] = 0;   // converged or non-finite: done for this colour class
  }
  if (a.out_local) a.out_local[s] = Lout;
}

__global__ __launch_bounds__(256) void k_skipped(const uint8_t* __restrict__ mask, int S, int32_t* status,
                                                 double* out_local) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= S || mask[s]) return;
  status[s] = CEL_ST_SKIPPED;
  if (out_local) out_local[s] = __longlong_as_double(0x7ff8000000000000LL);
}

// fills: radius <- r0 for all sources; active <- (colour == c) for one class
__global__ __launch_bounds__(256) void k_fill_radius(double* radius, int S, double r0) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s < S) radius[s] = r0;
}
__global__ __launch_bounds__(256) void k_set_active(uint8_t* active, const int32_t* __restrict__ colour, int S, int c) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s < S) active[s] = colour[s] == c ? 1 : 0;
}
__global__ __launch_bounds__(256) void k_count_active(const uint8_t* __restrict__ active, const int32_t* __restrict__ list,
                                                      int n, int32_t* out) {
  __shared__ int sh[256];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 256) c += active[list[i]];
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// One Newton iteration of colour class `cls` on the sources flagged in `active`.
static hipError_t enqueue_newton_class(cel_plan* p, double* theta, double* radius, uint8_t* active, int cls,
                                       int32_t* status, double* out_local, bool clear_done, hipStream_t sm) {
  const bool fp64 = p->opt.pixel_fp64 || p->opt.hessian_fp64;
  const int nsrc = (int)p->class_src[cls].size();
  if (nsrc == 0) return hipSuccess;
  // gradients at the iterate and at the 54 central-difference points
  hipError_t e = eval_any(p, theta, nullptr, 0, 2 * kParamN + 1, true, cls, active, sm, true, fp64);
  if (e != hipSuccess) return e;
  TrArgs ta;
  std::memset(&ta, 0, sizeof(ta));
  ta.job_src = p->d_class_src[cls];
  ta.n_jobs = nsrc;
  ta.S = p->S;
  ta.active = active;
  ta.v_grad = p->v_grad;
  ta.v_local = p->v_local;
  ta.fd_step = p->opt.fd_step;
  ta.theta = theta;
  ta.radius = radius;
  ta.npix = p->d_npix;
  ta.gtol = p->opt.gtol;
  ta.ftol = p->opt.ftol;
  ta.radius_min = p->opt.radius_min;
  ta.theta_trial = p->d_theta_trial;
  ta.trial_active = p->d_trial_active;
  ta.pred = p->d_pred;
  ta.pnorm = p->d_step_norm;
  ta.status = status;
  ta.prior = p->d_prior;
  hipLaunchKernelGGL(k_trsolve, dim3(nsrc), dim3(64), 0, sm, ta);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // objective at the trial points
  e = eval_any(p, theta, p->d_theta_trial, kVariants - 1, 1, false, cls, p->d_trial_active, sm, false, fp64);
  if (e != hipSuccess) return e;
  AcceptArgs aa;
  std::memset(&aa, 0, sizeof(aa));
  aa.job_src = p->d_class_src[cls];
  aa.n_jobs = nsrc;
  aa.active = active;
  aa.clear_done = clear_done ? 1 : 0;
  aa.trial_active = p->d_trial_active;
  aa.local0 = p->v_local;
  aa.local_trial = p->v_local + (int64_t)(kVariants - 1) * p->S;
  aa.pred = p->d_pred;
  aa.pnorm = p->d_step_norm;
  aa.theta = theta;
  aa.theta_trial = p->d_theta_trial;
  aa.radius = radius;
  aa.status = status;
  aa.out_local = out_local;
  aa.eta = p->opt.eta;
  aa.radius_max = p->opt.radius_max;
  hipLaunchKernelGGL(k_accept, dim3((nsrc + 63) / 64), dim3(64), 0, sm, aa);
  return hipGetLastError();
}

}  // namespace celmi

using namespace celmi;

static cel_status newton_scratch(cel_plan* p) {
  const bool fp64 = p->opt.pixel_fp64 || p->opt.hessian_fp64;
  cel_status st = ensure_variants(p, kVariants, fp64);
  if (st) return st;
  return ensure_newton(p);
}

extern "C" cel_status cel_newton_step(cel_ctx* ctx, const cel_plan* cplan, double* theta, double* radius,
                                      const uint8_t* mask, int32_t* step_status, double* elbo_local, void* stream) {
  if (!ctx || !cplan) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (p->S > 0 && (!theta || !radius || !step_status)) return CEL_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  // the stepped sources must be pairwise non-overlapping
  std::vector<uint8_t> m(p->S, 1);
  if (mask)
    for (int s = 0; s < p->S; ++s) m[s] = mask[s] ? 1 : 0;
  for (int s = 0; s < p->S; ++s)
    if (m[s])
      for (int t : p->adj[s])
        if (m[t]) return CEL_EINVAL;
  cel_status st = newton_scratch(p);
  if (st) return st;
  if (p->S == 0) return CEL_OK;
  // stage the mask through the plan's pinned buffer (wait for the previous copy first)
  if (hipEventSynchronize(p->mask_copied) != hipSuccess) return CEL_EHIP;
  std::memcpy(p->h_mask, m.data(), p->S);
  hipError_t e = hipMemcpyAsync(p->d_mask, p->h_mask, p->S, hipMemcpyHostToDevice, sm);
  if (e == hipSuccess) e = hipEventRecord(p->mask_copied, sm);
  for (int c = 0; c < p->n_colours && e == hipSuccess; ++c) {
    bool any = false;
    for (int s : p->class_src[c]) any = any || m[s];
    if (any) e = enqueue_newton_class(p, theta, radius, p->d_mask, c, step_status, elbo_local, false, sm);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_skipped, dim3((p->S + 255) / 256), dim3(256), 0, sm, p->d_mask, p->S, step_status,
                       elbo_local);
    e = hipGetLastError();
  }
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

extern "C" cel_status cel_sweep(cel_ctx* ctx, const cel_plan* cplan, double* theta, double* radius, int32_t* status,
                                const cel_sweep_opts* opts, cel_sweep_report* report, void* stream) {
  if (!ctx || !cplan) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (p->S > 0 && (!theta || !radius || !status)) return CEL_EINVAL;
  cel_sweep_opts o;
  o.n_sweeps = 3;
  o.max_newton_iters = 50;
  o.use_graph = 1;
  if (opts) {
    if (opts->n_sweeps < 0 || opts->max_newton_iters < 0) return CEL_EINVAL;
    o = *opts;
  }
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  cel_status st = newton_scratch(p);
  if (st) return st;
  // graphs cannot be captured on the null stream: run on the plan's own stream after the
  // caller's prior work, and synchronise before returning (the call is synchronous anyway)
  if (o.use_graph && sm == nullptr) {
    if (hipStreamSynchronize(sm) != hipSuccess) return CEL_EHIP;
    sm = p->own_stream;
  }
  const auto t0 = std::chrono::steady_clock::now();
  int64_t steps = 0;
  hipError_t e = hipSuccess;
  const int S = p->S;
  if (S > 0) {
    hipLaunchKernelGGL(k_set_active, dim3((S + 255) / 256), dim3(256), 0, sm, p->d_mask, p->d_colour, S, -1);
    e = hipGetLastError();
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_skipped, dim3((S + 255) / 256), dim3(256), 0, sm, p->d_mask, S, status, nullptr);
  }
  // one captured graph per colour class: a full Newton iteration of the class
  if (o.use_graph && p->graphs.size() != (size_t)p->n_colours) {
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.assign(p->n_colours, {});
  }
  const int check_every = 4;
  for (int sw = 0; sw < o.n_sweeps && e == hipSuccess && S > 0; ++sw) {
    hipLaunchKernelGGL(k_fill_radius, dim3((S + 255) / 256), dim3(256), 0, sm, radius, S, p->opt.radius0);
    if ((e = hipGetLastError()) != hipSuccess) break;
    for (int c = 0; c < p->n_colours && e == hipSuccess; ++c) {
      const int nsrc = (int)p->class_src[c].size();
      hipLaunchKernelGGL(k_set_active, dim3((S + 255) / 256), dim3(256), 0, sm, p->d_mask, p->d_colour, S, c);
      if ((e = hipGetLastError()) != hipSuccess) break;
      hipGraphExec_t exec = nullptr;
      if (o.use_graph) {
        auto& G = p->graphs[c];
        if (!G.exec || G.theta != theta || G.radius != radius || G.status != status || G.stream != sm) {
          if (G.exec) (void)hipGraphExecDestroy(G.exec);
          G.exec = nullptr;
          hipGraph_t graph;
          e = hipStreamBeginCapture(sm, hipStreamCaptureModeThreadLocal);
          if (e != hipSuccess) break;
          hipError_t e2 = enqueue_newton_class(p, theta, radius, p->d_mask, c, status, nullptr, true, sm);
          e = hipStreamEndCapture(sm, &graph);
          if (e2 != hipSuccess) e = e2;
          if (e != hipSuccess) break;
          e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          if (e != hipSuccess) break;
          G.theta = theta;
          G.radius = radius;
          G.status = status;
          G.stream = sm;
        }
        exec = G.exec;
      }
      for (int it = 0; it < o.max_newton_iters && e == hipSuccess; ++it) {
        if (exec) e = hipGraphLaunch(exec, sm);
        else e = enqueue_newton_class(p, theta, radius, p->d_mask, c, status, nullptr, true, sm);
        ++steps;
        if (e != hipSuccess) break;
        if ((it + 1) % check_every == 0 || it + 1 == o.max_newton_iters) {
          hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, sm, p->d_mask, p->d_class_src[c], nsrc,
                             p->d_counter);
          e = hipMemcpyAsync(p->h_counter, p->d_counter, sizeof(int32_t), hipMemcpyDeviceToHost, sm);
          if (e == hipSuccess) e = hipStreamSynchronize(sm);
          if (e != hipSuccess) break;
          if (*p->h_counter == 0) break;
        }
      }
    }
  }
  if (e == hipSuccess && S > 0) e = launch_total_after_eval(p, theta, sm);
  double tot = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(p->h_total, p->d_total, sizeof(double), hipMemcpyDeviceToHost, sm);
  if (e == hipSuccess) e = hipStreamSynchronize(sm);
  if (e == hipSuccess) tot = S > 0 ? *p->h_total : 0.0;
  if (report) {
    report->elbo_total = tot;
    report->n_colours = p->n_colours;
    report->n_newton_steps = steps;
    report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}
