// HIP kernels (gfx950) of the variational objective of arXiv 1803.00113.
//
// Pipeline of one evaluation (ELBO, Section 4.2, and its gradient):
//   k_prep_tables  per (variant, patch): theta -> mixture component table (FP64 math,
//                  stored in the pixel precision) -- light kernels of Section 2.1.2
//                  (equation hsi) convolved with the image PSF (Section 2.2.3), flux
//                  moments of equation conditional
//   k_fused        per work item (a run of <= chunk pixels of one patch): for every pixel
//                  the own source's mixture value and partial derivatives, every
//                  overlapping neighbour's value, E_q[lambda] and V_q[lambda] (equations
//                  conditional, vareq), the delta-method pixel term (equation
//                  eq:log_p_last, Section 4.2.2) and its adjoint coefficients; FP64 sums
//                  reduced across the wavefront into one slot row per work item
//   k_finalize     per source: fixed-order reduction of its slot rows, FP64 chain rule to
//                  the unconstrained parameters, KL_s and its gradient (equations eq:kl,
//                  kleq, the GMM colour bound and Supplement A) on a second wavefront
//   k_total        one workgroup: fixed-order sum of the per-source owned objectives
#include <math.h>

#include "device.h"
#include "kernels.h"
#include "pixmath.h"

namespace celmi {

// Parameters of variant v of a source: base theta, +/- h along one coordinate, trial, or the
// variant's own parameter array (vstride > 0).  (central differences only when fd != 0; the
// trial point is variant trial_v)
__device__ __forceinline__ void load_theta(const double* theta, const double* theta_trial, int64_t vstride, int s,
                                           int v, double h, double* th, int trial_v, int fd) {
  const double* src = (v == trial_v && theta_trial) ? theta_trial + (int64_t)s * kThetaN
                                                    : theta + (int64_t)v * vstride + (int64_t)s * kThetaN;
  // the perturbed coordinate is selected arithmetically so that th stays in registers
  const int kp = (fd && v >= 1 && v <= kParamN) ? v - 1 : -1;
  const int km = (fd && v > kParamN && v <= 2 * kParamN) ? v - 1 - kParamN : -1;
#pragma unroll
  for (int k = 0; k < kThetaN; ++k) th[k] = src[k] + (k == kp ? h : 0.0) - (k == km ? h : 0.0);
}

// Galaxy covariance Sigma_s = R^T diag(r^2, axis^2 r^2) R, R = [[c,-s],[s,c]] (Section 2.1.2)
__device__ __forceinline__ void galaxy_cov(double angle, double radius, double axis, double* sig) {
  double c = cos(angle), s = sin(angle), r2 = radius * radius, a2 = axis * axis;
  sig[0] = r2 * (c * c + a2 * s * s);
  sig[1] = r2 * (a2 - 1.0) * c * s;
  sig[2] = r2 * (s * s + a2 * c * c);
}

// ----------------------------------------------------------------------------------------
// k_prep_tables: one wavefront per (variant, patch)

template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void k_prep_tables(
    PrepArgs a) {
  const int pi_ = a.patch_list ? a.patch_list[blockIdx.x] : a.patch_offset + (int)blockIdx.x;
  const int v = a.variant0 + blockIdx.y;
  const DPatch P = a.patches[pi_];
  if (a.active && !a.active[P.src]) return;
  if (a.active_v && !a.active_v[(int64_t)blockIdx.y * a.active_v_stride + P.src]) return;
  const cel_image& im = a.images[P.img];
  double th[kThetaN];
  load_theta(a.theta, a.theta_trial, a.theta_vstride, P.src, v, a.fd_step, th, a.trial_variant, a.fd);
  Table<T>* tb = reinterpret_cast<Table<T>*>(a.tables) + (int64_t)v * a.n_patches + pi_;
  const int lane = threadIdx.x;
  // position in patch-local pixel coordinates: mu = A u + b - (x0, y0)
  const double mux = im.A[0][0] * th[0] + im.A[0][1] * th[1] + im.b[0] - P.x0;
  const double muy = im.A[1][0] * th[0] + im.A[1][1] * th[1] + im.b[1] - P.y0;
  // The source's exponentials are taken one per lane and broadcast, so that the exp code
  // runs once per wavefront instead of once per value: lanes 0-1 the flux variances, 2-9
  // the colour variances, 10 the radius, 11-13 exp(-x) of the type, axis and profile
  // logits (sigmoid(x) = 1 / (1 + exp(-x))).
  double earg = 0.0;
#pragma unroll
  for (int l = 0; l < 14; ++l) {
    const double x = l < 2 ? th[5 + l] : l < 10 ? th[15 + (l - 2)] : l == 10 ? th[24] : l == 11 ? -th[2]
                     : l == 12 ? -th[26] : -th[25];
    earg = lane == l ? x : earg;
  }
  double eval = exp(earg);
  if (lane >= 11 && lane <= 13) eval = 1.0 / (1.0 + eval);
  double ex[14];
#pragma unroll
  for (int l = 0; l < 14; ++l) ex[l] = __shfl(eval, l, 64);
  double sig[3];
  galaxy_cov(th[23], ex[10], ex[12], sig);
  // pixel-frame galaxy covariance S = A Sigma A^T
  const double a00 = im.A[0][0], a01 = im.A[0][1], a10 = im.A[1][0], a11 = im.A[1][1];
  const double t00 = a00 * sig[0] + a01 * sig[1], t01 = a00 * sig[1] + a01 * sig[2];
  const double t10 = a10 * sig[0] + a11 * sig[1], t11 = a10 * sig[1] + a11 * sig[2];
  const double Sxx = t00 * a00 + t01 * a01, Sxy = t00 * a10 + t01 * a11, Syy = t10 * a10 + t11 * a11;
  const int K = im.n_psf;
  // the PSF mixture of this patch: its own where the PSF varies over the image
  const double(*psf)[6] = a.patch_psf ? reinterpret_cast<const double(*)[6]>(a.patch_psf + (int64_t)pi_ * kMaxPsf * 6)
                                      : im.psf;
  // flux moments given the type (equation conditional): log l ~ N(m, v)
  const double aa = ex[11];
  const double w[2] = {1.0 - aa, aa};
  double m[2], var[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    m[i] = th[3 + i];
    var[i] = ex[i];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double W = c_W[im.band][c];
      m[i] += W * th[7 + 4 * i + c];
      var[i] += W * W * ex[2 + 4 * i + c];
    }
  }
  // lanes 0-1: exp(m + v/2); lanes 2-3: expm1(v); then broadcast
  const int li = lane & 1;
  const double mi = li ? m[1] : m[0], vi = li ? var[1] : var[0];
  const double ev2 = lane < 2 ? exp(mi + 0.5 * vi) : expm1(vi);
  double L[2], kk[2], ee[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    L[i] = im.iota * __shfl(ev2, i, 64);
    ee[i] = __shfl(ev2, 2 + i, 64);
    kk[i] = w[i] * L[i] * L[i] * ee[i];
  }
  // component cuts below scale with the flux: log2 of L0, L1 and the sky minimum, one per lane
  const double smin = a.sky_min ? a.sky_min[pi_] : 0.0;
  const double larg = lane == 0 ? L[0] : lane == 1 ? L[1] : smin;
  const double lg = log2(larg);
  const double cut_gal = density_cut_log2<T>(L[0], smin, __shfl(lg, 0, 64), __shfl(lg, 2, 64));
  const double cut_star = density_cut_log2<T>(L[1], smin, __shfl(lg, 1, 64), __shfl(lg, 2, 64));
  if (lane == 0) {
    tb->hdr[8] = (T)ee[0];
    tb->hdr[9] = (T)ee[1];
    tb->hdr[0] = (T)L[0];
    tb->hdr[1] = (T)L[1];
    tb->hdr[2] = (T)w[0];
    tb->hdr[3] = (T)w[1];
    tb->hdr[4] = (T)kk[0];
    tb->hdr[5] = (T)kk[1];
    tb->hdr[6] = (T)(w[0] * w[1]);
    tb->hdr[7] = (T)ex[13];
    tb->hdr[10] = (T)mux;
    tb->hdr[11] = (T)muy;
  }
  // components: 4 star slots then 4 x 16 galaxy slots
  for (int c = lane; c < kMaxPsf + kMaxPsf * 2 * kMaxProf; c += 64) {
    // a star slot (c < kMaxPsf) or a galaxy slot: the same 2x2 algebra, one code path
    const bool star = c < kMaxPsf;
    const int g = c - kMaxPsf;
    const int k = star ? c : g / (2 * kMaxProf), j = star ? 0 : g % (2 * kMaxProf);
    const bool isdev = j >= kMaxProf;
    const int jj = isdev ? j - kMaxProf : j;
    const int nj = isdev ? a.prof->n_dev : a.prof->n_exp;
    const bool used = k < K && (star || jj < nj);
    double tau = 0.0, Pxx = 0.0, Pxy = 0.0, Pyy = 0.0, lw = kNegHuge, rc2 = -1.0;
    if (used) {   // (an iteration whose slots are all unused skips the math)
      const int pj = isdev ? a.prof->n_exp + jj : jj;
      tau = star ? 0.0 : a.prof->tau[pj];
      const double alpha = star ? 1.0 : a.prof->alpha[pj];
      const double cxx = psf[k][3] + tau * Sxx, cxy = psf[k][4] + tau * Sxy, cyy = psf[k][5] + tau * Syy;
      const double det = cxx * cyy - cxy * cxy, rdet = 1.0 / det;
      const double wt = psf[k][0] * alpha;
      Pxx = cyy * rdet;
      Pxy = -cxy * rdet;
      Pyy = cxx * rdet;
      // log2 of weight / (2 pi sqrt(det))
      lw = wt > 0 ? log2(wt * sqrt(rdet)) - kLog2TwoPi : kNegHuge;
      rc2 = cut_radius2(lw, cxx, cxy, cyy, star ? cut_star : cut_gal);
    }
    const double hl = -0.5 * kLog2e;
    const T qv[4] = {(T)(hl * Pxx), (T)(hl * Pxy), (T)(hl * Pyy), (T)lw};
    const T pv[3] = {(T)Pxx, (T)Pxy, (T)Pyy};
    if (star) {
      T* r = tb->star[k];
      const double ox = used ? psf[k][1] : 0.0, oy = used ? psf[k][2] : 0.0;
      r[0] = (T)(used ? mux + ox : 0.0);
      r[1] = (T)(used ? muy + oy : 0.0);
      r[2] = pv[0];
      r[3] = pv[1];
      r[4] = pv[2];
      r[5] = (T)lw;
      r[6] = r[7] = (T)0;
      tb->rc2s[k] = (T)rc2 + (T)0;   // (+ 0: a -0 becomes +0, for the integer-ordered cut test)
#pragma unroll
      for (int e = 0; e < 4; ++e) tb->sq[k][e] = qv[e];
      if (a.records & kRecRuns) tb->rq[k][0] = (T)exp(-Pxx);
    } else {
      tb->rc2[k][j] = (T)rc2 + (T)0;
      if (a.records & kRecRuns) tb->rq[k][1 + j] = (T)exp(-Pxx);
#pragma unroll
      for (int e = 0; e < 4; ++e) tb->gq[k][j][e] = qv[e];
      const double c2 = kExpScale * kExpScale;
      T* gs = tb->gq[k][j] + 4;
      gs[0] = (T)(c2 * Pxx);
      gs[1] = (T)(c2 * Pxy);
      gs[2] = (T)(c2 * Pyy);
      gs[3] = (T)(0.5 * tau);
      if (!(a.records & kRecHessian)) continue;
      T* r = tb->gal[k][j];
      r[0] = pv[0];
      r[1] = pv[1];
      r[2] = pv[2];
      r[3] = (T)lw;
      const double h = 0.5 * tau * tau;
      T* q = tb->gt[k][j];
      q[0] = (T)tau;
      q[1] = (T)(tau * tau);
      q[2] = (T)(h * Pxx * Pxx);
      q[3] = (T)(h * 2.0 * Pxx * Pxy);
      q[4] = (T)(h * Pxy * Pxy);
      q[5] = (T)(h * (2.0 * Pxy * Pxy + 2.0 * Pxx * Pyy));
      q[6] = (T)(h * 2.0 * Pxy * Pyy);
      q[7] = (T)(h * Pyy * Pyy);
    }
  }
}

// ----------------------------------------------------------------------------------------
// k_fused: the per-pixel hot loop

// Copy the galaxy components' exponent records of the K PSF components of one table into
// LDS (one wavefront; 16-byte vectors).  Each component's record is then one broadcast LDS
// read rather than a scalar-cache load: the tables of the wavefronts resident on a compute
// unit exceed its scalar cache.
template <typename T>
__device__ __forceinline__ void stage_records(const Table<T>* __restrict__ tb, int K, int lane,
                                              T (*rec)[2 * kMaxProf][8]) {
  constexpr int kVec = 16 / sizeof(T);   // values per 16-byte vector
  const int n = K * 2 * kMaxProf * 8 / kVec;
  const uint4* src = reinterpret_cast<const uint4*>(&tb->gq[0][0][0]);
  uint4* dst = reinterpret_cast<uint4*>(&rec[0][0][0]);
  for (int i = lane; i < n; i += 64) dst[i] = src[i];
  __syncthreads();
}

// Values of a source's star (f1) and galaxy (f0) light at PPL pixels (local coords of the
// source's own patch).  Neighbour evaluation: no derivatives.  A type of weight exactly 0
// (a point value of the type) is not evaluated: its light enters the moments only through
// that weight.
template <typename T, int PPL, int NEXP, int NDEV>
__device__ __forceinline__ void eval_values(const Table<T>* __restrict__ tb, const T (*__restrict__ rec)[2 * kMaxProf][8],
                                            int K, const T* px, const T* py, const T* box, T* f0, T* f1) {
  T fe[PPL], fd[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) fe[i] = fd[i] = f1[i] = (T)0;
  const bool use_gal = tb->hdr[2] != (T)0, use_star = tb->hdr[3] != (T)0;
  for (int k = 0; k < K; ++k) {
    const T mx = tb->star[k][0], my = tb->star[k][1];
    T dx[PPL], dy[PPL], xx[PPL], xy[PPL], yy[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      dx[i] = px[i] - mx;
      dy[i] = py[i] - my;
      xx[i] = dx[i] * dx[i];
      xy[i] = (T)2 * dx[i] * dy[i];
      yy[i] = dy[i] * dy[i];
    }
    const T d2 = box_dist2<T>(mx, my, box);
    // this PSF component's cut radii, read before any is used (one wait for all of them
    // instead of one per component); the exponent records come from the LDS copy
    T rc[NEXP + NDEV];
#pragma unroll
    for (int j = 0; j < NEXP + NDEV; ++j) rc[j] = tb->rc2[k][j < NEXP ? j : kMaxProf + (j - NEXP)];
    // a type of weight 0 sees its components at infinite distance: all skipped
    const auto d2s = uniform_cut_key(use_star ? d2 : (T)INFINITY), d2g = uniform_cut_key(use_gal ? d2 : (T)INFINITY);
    if (!(d2s > cut_key(tb->rc2s[k]))) {
#pragma unroll
      for (int i = 0; i < PPL; ++i) f1[i] += comp_value<T>(tb->sq[k], xx[i], xy[i], yy[i]);
    }
#pragma unroll
    for (int j = 0; j < NEXP; ++j) {
      if (d2g > cut_key(rc[j])) continue;
#pragma unroll
      for (int i = 0; i < PPL; ++i) fe[i] += comp_value<T>(rec[k][j], xx[i], xy[i], yy[i]);
    }
#pragma unroll
    for (int j = 0; j < NDEV; ++j) {
      if (d2g > cut_key(rc[NEXP + j])) continue;
#pragma unroll
      for (int i = 0; i < PPL; ++i) fd[i] += comp_value<T>(rec[k][kMaxProf + j], xx[i], xy[i], yy[i]);
    }
  }
  const T pi = tb->hdr[7];
#pragma unroll
  for (int i = 0; i < PPL; ++i) f0[i] = pi * fd[i] + ((T)1 - pi) * fe[i];
}

// Own source: values and partial derivatives w.r.t. the pixel-frame centre mu, the
// pixel-frame galaxy covariance S and the profile weight.  For N = weight * normal(p; m, C)
// with P = C^{-1}, u = P (p - m):  dN/dmu = N u,  dN/dC = N (u u^T - P) / 2,  dC/dS = tau.
// The records hold c P with c = -log2(e)/2 (gq, sq), so the lanes form u' = c u and the
// exponent d . u' + log2 weight directly; the sums g = sum N u' and s = sum tau/2 N (u' u'^T
// - c^2 P) are c and c^2 times the plain derivatives (divided back per slot row).
template <typename T, int PPL>
struct OwnPix {
  T f1[PPL], g1x[PPL], g1y[PPL];
  T fe[PPL], gex[PPL], gey[PPL], sexx[PPL], sexy[PPL], seyy[PPL];
  T fd[PPL], gdx[PPL], gdy[PPL], sdxx[PPL], sdxy[PPL], sdyy[PPL];
};

// MODE 0: value only; 1: value and d/dmu; 2: value, d/dmu and d/dS.  q: (c P_xx, c P_xy,
// c P_yy, log2 weight); r (MODE 2): (c^2 P_xx, c^2 P_xy, c^2 P_yy, tau/2)
template <typename T, int PPL, int MODE>
__device__ __forceinline__ void comp_own(const T* __restrict__ q, const T* __restrict__ r, const T* dx, const T* dy,
                                         T* f, T* gx, T* gy, T* sxx, T* sxy, T* syy) {
  const T q0 = q[0], q1 = q[1], q2 = q[2], lw = q[3];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const T ux = fma(q0, dx[i], q1 * dy[i]);
    const T uy = fma(q1, dx[i], q2 * dy[i]);
    const T N = fexp2<T>(fma(dx[i], ux, fma(dy[i], uy, lw)));
    f[i] += N;
    if (MODE >= 1) {
      gx[i] = fma(N, ux, gx[i]);
      gy[i] = fma(N, uy, gy[i]);
    }
    if (MODE >= 2) {
      const T tN = r[3] * N;
      sxx[i] = fma(tN, fma(ux, ux, -r[0]), sxx[i]);
      sxy[i] = fma(tN, fma(ux, uy, -r[1]), sxy[i]);
      syy[i] = fma(tN, fma(uy, uy, -r[2]), syy[i]);
    }
  }
}

// The own source's values (and, with DERIV, partial derivatives).  The values are formed
// by the same operations with or without DERIV, so the ELBO-only and the gradient paths
// give bitwise-identical objectives.  Without DERIV a type of weight exactly 0 (a point
// value of the type) is not evaluated: its light enters the moments only through that
// weight, so the objective is unchanged.
template <typename T, int PPL, int NEXP, int NDEV, bool DERIV>
__device__ __forceinline__ void eval_own(const Table<T>* __restrict__ tb, const T (*__restrict__ rec)[2 * kMaxProf][8],
                                         int K, const T* px, const T* py, const T* box, OwnPix<T, PPL>& o) {
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    o.f1[i] = o.g1x[i] = o.g1y[i] = (T)0;
    o.fe[i] = o.gex[i] = o.gey[i] = o.sexx[i] = o.sexy[i] = o.seyy[i] = (T)0;
    o.fd[i] = o.gdx[i] = o.gdy[i] = o.sdxx[i] = o.sdxy[i] = o.sdyy[i] = (T)0;
  }
  __builtin_assume(K >= 1);   // images have 1..kMaxPsf PSF components (checked at prepare)
  const bool use_gal = DERIV || tb->hdr[2] != (T)0, use_star = DERIV || tb->hdr[3] != (T)0;
  for (int k = 0; k < K; ++k) {
    const T mx = tb->star[k][0], my = tb->star[k][1];
    T dx[PPL], dy[PPL], z[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) z[i] = (T)0;
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      dx[i] = px[i] - mx;
      dy[i] = py[i] - my;
    }
    const T d2 = box_dist2<T>(mx, my, box);
    // this PSF component's cut radii, read before any is used: one wait for all of them
    // instead of a scalar load and its wait ahead of each component
    T rc[NEXP + NDEV];
#pragma unroll
    for (int j = 0; j < NEXP + NDEV; ++j) rc[j] = tb->rc2[k][j < NEXP ? j : kMaxProf + (j - NEXP)];
    const T rcs = tb->rc2s[k];
    // a type of weight 0 sees its components at infinite distance: all skipped
    const auto d2s = uniform_cut_key(use_star ? d2 : (T)INFINITY), d2g = uniform_cut_key(use_gal ? d2 : (T)INFINITY);
    if (!(d2s > cut_key(rcs)))
      comp_own<T, PPL, DERIV ? 1 : 0>(tb->sq[k], nullptr, dx, dy, o.f1, o.g1x, o.g1y, z, z, z);
#pragma unroll
    for (int j = 0; j < NEXP; ++j)
      if (!(d2g > cut_key(rc[j])))
        comp_own<T, PPL, DERIV ? 2 : 0>(rec[k][j], rec[k][j] + 4, dx, dy, o.fe, o.gex, o.gey, o.sexx, o.sexy,
                                        o.seyy);
#pragma unroll
    for (int j = 0; j < NDEV; ++j)
      if (!(d2g > cut_key(rc[NEXP + j])))
        comp_own<T, PPL, DERIV ? 2 : 0>(rec[k][kMaxProf + j], rec[k][kMaxProf + j] + 4, dx, dy, o.fd, o.gdx,
                                        o.gdy, o.sdxx, o.sdxy, o.sdyy);
  }
}

// k_maps: every source's own moments E_s, V_s (values only) on its patches' overlap boxes at
// the base parameters, read by the pixel kernel for overlapping neighbours.
template <typename T, int PPL, int NEXP, int NDEV>
__global__ __launch_bounds__(64) void k_maps(MapArgs a) {
  const int pos = xcd_position((int)blockIdx.x, (int)gridDim.x);
  const DMapTask task = a.tasks[pos];
  const DPatch P = a.patches[task.patch];
  const Table<T>* __restrict__ tb = reinterpret_cast<const Table<T>*>(a.base) + task.patch;
  const int K = a.img_npsf[P.img];
  const int lane = threadIdx.x;
  const T L0 = tb->hdr[0], L1 = tb->hdr[1], w0 = tb->hdr[2], w1 = tb->hdr[3];
  const T k0 = tb->hdr[4], k1 = tb->hdr[5], w01 = tb->hdr[6];
  __shared__ T rec[kMaxPsf][2 * kMaxProf][8];
  stage_records<T>(tb, K, lane, rec);
  // box-local coordinates of this lane's pixels, advanced by a carry per group (patch-local:
  // plus the box corner)
  const int bw = task.w;
  const int step = 64 * PPL;
  const int step_rows = step / bw, step_cols = step - step_rows * bw;
  int col[PPL], row[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int idx = task.pix_begin + i * 64 + lane;
    row[i] = idx / bw;
    col[i] = idx - row[i] * bw;
  }
  for (int base = task.pix_begin; base < task.pix_end; base += step) {
    T px[PPL], py[PPL], f0[PPL], f1[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      px[i] = (T)(col[i] + task.x0);
      py[i] = (T)(row[i] + task.y0);
    }
    int ibox[4];
    run_box<int>(base, min(base + step, task.pix_end), bw, ibox);
    const T box[4] = {(T)(ibox[0] + task.x0), (T)(ibox[1] + task.x0), (T)(ibox[2] + task.y0),
                      (T)(ibox[3] + task.y0)};
    eval_values<T, PPL, NEXP, NDEV>(tb, rec, K, px, py, box, f0, f1);
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int idx = base + i * 64 + lane;
      if (idx >= task.pix_end) continue;
      const T a0 = L0 * f0[i], a1 = L1 * f1[i], d = a0 - a1;
      const T Es = w0 * a0 + w1 * a1;
      const T Vs = fma(k0 * f0[i], f0[i], fma(k1 * f1[i], f1[i], w01 * d * d));
      const int64_t at = P.off + (int64_t)(row[i] + task.y0) * P.w + col[i] + task.x0;
      if constexpr (sizeof(T) == 8)
        reinterpret_cast<double2*>(a.maps)[at] = make_double2(Es, Vs);
      else
        reinterpret_cast<float2*>(a.maps)[at] = make_float2(Es, Vs);
    }
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      col[i] += step_cols;
      row[i] += step_rows;
      if (col[i] >= bw) {
        col[i] -= bw;
        row[i] += 1;
      }
    }
  }
}

// Values of one mixture component over a run of kRun consecutive pixels of one row,
// accumulated into acc[0..kRun): x0 the first pixel's column offset from the component's
// centre, dy the row offset, q = (q0, q1, q2, log2 weight) its exponent record, c = 2^(2 q0).
// The exponent is quadratic along the row, so the value is advanced by the ratio
// r(x) = 2^(q(x+1) - q(x)), and r by the constant factor c: two products per pixel instead of
// an exponent and an exponential.  The first value is the direct one; a first value below
// 2^-100 is formed 2^64 larger and scaled back as it is accumulated, so that a run rising
// towards the centre never starts from an underflowed value.
constexpr int kRun = 8;
template <typename T>
__device__ __forceinline__ void comp_run(const T* __restrict__ q, T c, T x0, T dy, T* acc) {
  const T e0 = fma(q[0], x0 * x0, fma(q[1], (T)2 * x0 * dy, fma(q[2], dy * dy, q[3])));
  const bool low = e0 < (T)-100;
  T v = fexp2<T>(low ? e0 + (T)64 : e0);
  const T scale = low ? (T)5.42101086242752217e-20 : (T)1;   // 2^-64
  T r = fexp2<T>(fma(q[0], fma((T)2, x0, (T)1), (T)2 * q[1] * dy));
  acc[0] = fma(v, scale, acc[0]);
#pragma unroll
  for (int k = 1; k < kRun; ++k) {
    v *= r;
    r *= c;
    acc[k] = fma(v, scale, acc[k]);
  }
}

// k_maps_runs: the same moments as k_maps, each lane taking a run of up to kRun consecutive
// pixels of one row of the work item (runs are cut at row ends), values by recurrence along
// the run.  Runs of one row: ceil(row length / kRun); the work item's rows: a partial first
// row, full rows, a partial last row.
template <typename T, int NEXP, int NDEV>
__global__ __launch_bounds__(64) void k_maps_runs(MapArgs a) {
  const int pos = xcd_position((int)blockIdx.x, (int)gridDim.x);
  const DMapTask task = a.tasks[pos];
  const DPatch P = a.patches[task.patch];
  const Table<T>* __restrict__ tb = reinterpret_cast<const Table<T>*>(a.base) + task.patch;
  const int K = a.img_npsf[P.img];
  const int lane = threadIdx.x;
  const T L0 = tb->hdr[0], L1 = tb->hdr[1], w0 = tb->hdr[2], w1 = tb->hdr[3];
  const T k0 = tb->hdr[4], k1 = tb->hdr[5], w01 = tb->hdr[6], pi = tb->hdr[7];
  const bool use_gal = tb->hdr[2] != (T)0, use_star = tb->hdr[3] != (T)0;
  // rows and columns below are local to the overlap box (w wide at (bx, by) in the patch)
  const int w = task.w, pb = task.pix_begin, pe = task.pix_end, bx = task.x0, by = task.y0;
  if (pe <= pb) return;
  const int r0 = pb / w, r1 = (pe - 1) / w;
  const int c_first = pb - r0 * w;
  const int len_first = r0 == r1 ? pe - pb : w - c_first;
  const int n_first = (len_first + kRun - 1) / kRun;
  const int per_row = (w + kRun - 1) / kRun;
  const int n_mid = r1 > r0 + 1 ? (r1 - r0 - 1) * per_row : 0;
  const int len_last = r0 == r1 ? 0 : pe - r1 * w;
  const int n_runs = n_first + n_mid + (len_last + kRun - 1) / kRun;
  T box[4];
  run_box<T>(pb, pe, w, box);   // the whole work item (one pass or several)
  box[0] += (T)bx;
  box[1] += (T)bx;
  box[2] += (T)by;
  box[3] += (T)by;
  for (int g0 = 0; g0 < n_runs; g0 += 64) {
    const int g = g0 + lane;
    int row, col0, len;
    if (g < n_first) {
      row = r0;
      col0 = c_first + kRun * g;
      len = min(kRun, len_first - kRun * g);
    } else if (g < n_first + n_mid) {
      const int h = g - n_first, rr = h / per_row, sgm = h - rr * per_row;
      row = r0 + 1 + rr;
      col0 = kRun * sgm;
      len = min(kRun, w - kRun * sgm);
    } else {
      const int sgm = g - n_first - n_mid;
      row = r1;
      col0 = kRun * sgm;
      len = min(kRun, len_last - kRun * sgm);
    }
    if (g >= n_runs) len = 0;
    T fe[kRun], fd[kRun], f1[kRun];
#pragma unroll
    for (int i = 0; i < kRun; ++i) fe[i] = fd[i] = f1[i] = (T)0;
    for (int k = 0; k < K; ++k) {
      const T mx = tb->star[k][0], my = tb->star[k][1];
      const T x0 = (T)(col0 + bx) - mx, dy = (T)(row + by) - my;
      const T d2 = box_dist2<T>(mx, my, box);
      const auto d2s = uniform_cut_key(use_star ? d2 : (T)INFINITY), d2g = uniform_cut_key(use_gal ? d2 : (T)INFINITY);
      if (!(d2s > cut_key(tb->rc2s[k]))) comp_run<T>(tb->sq[k], tb->rq[k][0], x0, dy, f1);
#pragma unroll
      for (int j = 0; j < NEXP; ++j)
        if (!(d2g > cut_key(tb->rc2[k][j]))) comp_run<T>(tb->gq[k][j], tb->rq[k][1 + j], x0, dy, fe);
#pragma unroll
      for (int j = 0; j < NDEV; ++j)
        if (!(d2g > cut_key(tb->rc2[k][kMaxProf + j])))
          comp_run<T>(tb->gq[k][kMaxProf + j], tb->rq[k][1 + kMaxProf + j], x0, dy, fd);
    }
    const int64_t at = P.off + (int64_t)(row + by) * P.w + col0 + bx;
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
      if (i >= len) break;
      const T f0 = pi * fd[i] + ((T)1 - pi) * fe[i];
      const T a0 = L0 * f0, a1 = L1 * f1[i], d = a0 - a1;
      const T Es = w0 * a0 + w1 * a1;
      const T Vs = fma(k0 * f0, f0, fma(k1 * f1[i], f1[i], w01 * d * d));
      if constexpr (sizeof(T) == 8)
        reinterpret_cast<double2*>(a.maps)[at + i] = make_double2(Es, Vs);
      else
        reinterpret_cast<float2*>(a.maps)[at + i] = make_float2(Es, Vs);
    }
  }
}

template <typename T, int PPL, bool GRAD, int NEXP, int NDEV>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && PPL < 4 ? 6 : 1))) void k_fused(
    FusedArgs<T> a) {
  const int v = a.variant0 + blockIdx.y;
  const int wi = a.order_offset + xcd_position((int)blockIdx.x, (int)gridDim.x);
  const int t = a.order ? a.order[wi] : wi;
  const DTask task = a.tasks[t];
  const DPatch P = a.patches[task.patch];
  if (a.active && !a.active[P.src]) return;
  if (a.active_v && !a.active_v[(int64_t)blockIdx.y * a.active_v_stride + P.src]) return;
  const Table<T>* __restrict__ tb = a.own + (int64_t)v * a.variant_stride + task.patch;
  const int K = a.img_npsf[P.img];
  const int lane = threadIdx.x;
  // the galaxy components' records of this patch, staged in LDS once per work item
  __shared__ T rec[kMaxPsf][2 * kMaxProf][8];
  stage_records<T>(tb, K, lane, rec);
  const T L0 = tb->hdr[0], L1 = tb->hdr[1], w0 = tb->hdr[2], w1 = tb->hdr[3];
  const T k0 = tb->hdr[4], k1 = tb->hdr[5], w01 = tb->hdr[6], pi = tb->hdr[7];
  // objective sums in FP64 per lane.  The 11 gradient sums are kept per lane in the pixel
  // precision over at most kFlush pixel groups, then summed over the wavefront in FP64 into
  // the work item's slot row (so a lane's partial sum never spans more than kFlush * PPL
  // pixels, whatever the chunk size)
  constexpr int kFlush = 4;
  double acc_t = 0.0, acc_own = 0.0;
  T part[S_T];
#pragma unroll
  for (int q = 0; q < S_T; ++q) part[q] = (T)0;
  double* out = a.slots + (int64_t)blockIdx.y * a.slot_variant_stride + (int64_t)t * kSlots;
  // patch-local coordinates of this lane's pixels, advanced by 64*PPL pixels per group:
  // one integer division at the start, then a carry
  const int step = 64 * PPL;
  const int step_rows = step / P.w, step_cols = step - step_rows * P.w;
  T px[PPL], py[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int idx = task.pix_begin + i * 64 + lane;
    const int row = idx / P.w;
    px[i] = (T)(idx - row * P.w);
    py[i] = (T)row;
  }
  const T wT = (T)P.w, srT = (T)step_rows, scT = (T)step_cols;
  int group = 0;

  for (int base = task.pix_begin; base < task.pix_end; base += step, ++group) {
    T xv[PPL], sky[PPL];
    bool valid[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      int idx = base + i * 64 + lane;
      valid[i] = idx < task.pix_end;
      if (!valid[i]) idx = task.pix_begin;
      if constexpr (sizeof(T) == 8) {
        const double2 xs = reinterpret_cast<const double2*>(a.xs)[P.off + idx];
        xv[i] = (T)xs.x;
        sky[i] = (T)xs.y;
      } else {
        const float2 xs = reinterpret_cast<const float2*>(a.xs)[P.off + idx];
        xv[i] = (T)xs.x;
        sky[i] = (T)xs.y;
      }
    }
    // own source
    T f0[PPL], f1[PPL];
    OwnPix<T, PPL> o;
    int ibox[4];
    run_box<int>(base, min(base + step, task.pix_end), P.w, ibox);
    const T box[4] = {(T)ibox[0], (T)ibox[1], (T)ibox[2], (T)ibox[3]};
    eval_own<T, PPL, NEXP, NDEV, GRAD>(tb, rec, K, px, py, box, o);
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      f1[i] = o.f1[i];
      f0[i] = fma(pi, o.fd[i], ((T)1 - pi) * o.fe[i]);
    }
    T E[PPL], V[PPL], d[PPL];
    bool own[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const T a0 = L0 * f0[i], a1 = L1 * f1[i];
      d[i] = a0 - a1;
      E[i] = sky[i] + w0 * a0 + w1 * a1;
      V[i] = fma(k0 * f0[i], f0[i], fma(k1 * f1[i], f1[i], w01 * d[i] * d[i]));
      own[i] = true;
    }
    // neighbours whose patch in this image covers the pixel (Section 2.2.3: the rate sums
    // over sources): their moments E_t, V_t at the pixel come from the per-patch maps.  A
    // neighbour whose rectangle misses the wavefront's pixel box is skipped as a whole.
    int ix[PPL], iy[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      ix[i] = (int)px[i];
      iy[i] = (int)py[i];
    }
    for (int nb = P.nbr_begin; nb < P.nbr_end; ++nb) {
      const DPatch Q = a.patches[a.nbr_idx[nb]];
      const int ox = P.x0 - Q.x0, oy = P.y0 - Q.y0;
      if (ibox[0] + ox >= Q.w || ibox[1] + ox < 0 || ibox[2] + oy >= Q.h || ibox[3] + oy < 0) continue;
      const bool lower = Q.src < P.src;
      const int64_t qoff = Q.off;
#pragma unroll
      for (int i = 0; i < PPL; ++i) {
        const int cx = ix[i] + ox, cy = iy[i] + oy;
        const bool in = valid[i] && (unsigned)cx < (unsigned)Q.w && (unsigned)cy < (unsigned)Q.h;
        if (in) {
          const int64_t at = qoff + (cy * Q.w + cx);
          if constexpr (sizeof(T) == 8) {
            const double2 ev = reinterpret_cast<const double2*>(a.maps)[at];
            E[i] += (T)ev.x;
            V[i] += (T)ev.y;
          } else {
            const float2 ev = reinterpret_cast<const float2*>(a.maps)[at];
            E[i] += (T)ev.x;
            V[i] += (T)ev.y;
          }
          if (lower) own[i] = false;
        }
      }
    }
    // pixel term (centred: the data constant x log x - x - log x! is added per patch in
    // FP64) and adjoint coefficients
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const T x = xv[i];
      const T invE = frcp<T>(E[i]);
      const T xr = x * invE * invE;
      T Tm = (x > (T)0 ? x_log_ratio<T>(x, E[i]) : (T)0) - (E[i] - x) - (T)0.5 * xr * V[i];
      if (!valid[i]) Tm = (T)0;
      acc_t += (double)Tm;
      acc_own += own[i] ? (double)Tm : 0.0;
      if (GRAD) {
        T cE = fma(xr * invE, V[i], (x - E[i]) * invE);
        T cV = (T)-0.5 * xr;
        if (!valid[i]) cE = cV = (T)0;
        const T rho0 = cE * w0 * L0 + (T)2 * cV * fma(k0, f0[i], w01 * L0 * d[i]);
        const T rho1 = cE * w1 * L1 + (T)2 * cV * fma(k1, f1[i], -w01 * L1 * d[i]);
        const T omp = (T)1 - pi;
        const T g0x = pi * o.gdx[i] + omp * o.gex[i], g0y = pi * o.gdy[i] + omp * o.gey[i];
        const T s0xx = pi * o.sdxx[i] + omp * o.sexx[i];
        const T s0xy = (T)2 * (pi * o.sdxy[i] + omp * o.sexy[i]);
        const T s0yy = pi * o.sdyy[i] + omp * o.seyy[i];
        const T cVf0 = cV * f0[i], cVf1 = cV * f1[i];
        part[S_CE_F0] = fma(cE, f0[i], part[S_CE_F0]);
        part[S_CE_F1] = fma(cE, f1[i], part[S_CE_F1]);
        part[S_CV_F00] = fma(cVf0, f0[i], part[S_CV_F00]);
        part[S_CV_F11] = fma(cVf1, f1[i], part[S_CV_F11]);
        part[S_CV_F01] = fma(cVf0, f1[i], part[S_CV_F01]);
        part[S_MU_X] = fma(rho0, g0x, fma(rho1, o.g1x[i], part[S_MU_X]));
        part[S_MU_Y] = fma(rho0, g0y, fma(rho1, o.g1y[i], part[S_MU_Y]));
        part[S_S_XX] = fma(rho0, s0xx, part[S_S_XX]);
        part[S_S_XY] = fma(rho0, s0xy, part[S_S_XY]);
        part[S_S_YY] = fma(rho0, s0yy, part[S_S_YY]);
        part[S_PI] = fma(rho0, o.fd[i] - o.fe[i], part[S_PI]);
      }
    }
    if (GRAD && (group % kFlush == kFlush - 1 || base + step >= task.pix_end)) {
      const bool first = group < kFlush;
      // the 11 wavefront sums together, then lane 0 reads each from the lane holding it and
      // stores it scaled back (the centre sums carry the records' scale c, the covariance
      // sums c^2); no per-lane slot index or address lives across the pixel loop
      const double sq = wave_sums<S_T, 32, T>(part, lane);
      // (the factors come with the kernel arguments, in scalar registers: no vector registers
      // hold them across the pixel loop)
      const double* unscale = a.unscale;
#pragma unroll
      for (int q = 0; q < S_T; ++q) {
        part[q] = (T)0;
        const double s = read_lane(sq, wave_sums_lane<S_T>(q));
        const double v = (q == S_MU_X || q == S_MU_Y) ? s * unscale[0]
                         : (q == S_S_XX || q == S_S_XY || q == S_S_YY) ? s * unscale[1] : s;
        if (lane == 0) out[q] = first ? v : out[q] + v;
      }
    }
    // next group: advance each lane's coordinates by step pixels
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      T c = px[i] + scT, r = py[i] + srT;
      if (c >= wT) {
        c -= wT;
        r += (T)1;
      }
      px[i] = c;
      py[i] = r;
    }
  }
  const double acc[2] = {acc_t, acc_own};
  const double s_t = wave_sums<2>(acc, lane);   // lane 0: the pixel term, lane 32: the owned part
  const int tslot = wave_sums_slot<2>(lane);
  if (tslot >= 0) out[S_T + tslot] = s_t;
  if (GRAD && task.pix_begin >= task.pix_end && lane == 0)
    for (int q = 0; q < S_T; ++q) out[q] = 0.0;
}

// ----------------------------------------------------------------------------------------
// k_finalize: per (variant, source) a wavefront whose lanes take the source's patches,
// partial sums combined in a fixed pairing, lane 0 applying the shape chain rule.  The KL
// term and its gradient do not depend on the pixels: launched with two wavefronts per
// block (small grids, where the kernel's time is one block's latency), the second evaluates
// them meanwhile and hands them over in LDS; with one (large grids, where two wavefronts
// per block would halve the blocks resident per compute unit) the first evaluates them
// after its sums.  Either way the same operations give the same numbers.
constexpr int kRed = 2 + kParamN + 3 + 1;   // pixel term, owned part, gradient, S gradient, profile
__global__ __launch_bounds__(128) void k_finalize(FinalizeArgs a) {
  const int jj = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const bool split = blockDim.x > 64, kl_wave = threadIdx.x >= 64;
  const int s = a.job_src ? a.job_src[jj] : jj + a.src_offset;
  const int vv = blockIdx.y;
  const int v = a.variant0 + vv;
  if (a.active && !a.active[s]) return;
  if (a.active_v && !a.active_v[(int64_t)vv * a.active_v_stride + s]) return;
  double th[kThetaN];
  load_theta(a.theta, a.theta_trial, a.theta_vstride, s, v, a.fd_step, th, a.trial_variant, a.fd);
  // the central-difference variants (1..54) carry the pixel part of the gradient only: the
  // KL part of the Hessian is taken analytically by the trust-region kernel
  const bool fd_variant = a.fd && v >= 1 && v <= 2 * kParamN;
  // the lanes' partial sums (first wavefront) and the KL value and its gradient, negated
  // (second wavefront)
  __shared__ double red[kRed], klg[1 + kParamN];
  double g[kThetaN];
  #pragma unroll
  for (int k = 0; k < kThetaN; ++k) g[k] = 0.0;
  double local = 0, own = 0, gS[3] = {0, 0, 0}, gpi = 0;
  const double ang = th[23], rad = exp(th[24]), prof = sigmoid(th[25]), axis = sigmoid(th[26]);
  double sig[3];
  // KL by the whole wavefront; its gradient is subtracted from zeros and added to the pixel
  // gradient below (a - b and a + (0 - b) are the same number)
  auto kl_to_lds = [&](double* gk) {
    const double kl = a.no_kl ? 0.0 : kl_source_wave(*a.prior, th, gk, fd_variant ? 0.0 : 1.0, lane);
    if (lane == 0) {
      klg[0] = kl;
      #pragma unroll
      for (int k = 0; k < kParamN; ++k) klg[1 + k] = gk[k];
    }
  };
  if (kl_wave) {
    kl_to_lds(g);
  } else {
    const double aa = sigmoid(th[2]);
    const double w0 = 1.0 - aa, w1 = aa;
    galaxy_cov(ang, rad, axis, sig);
    const double* slots = a.slots + (int64_t)vv * a.slot_variant_stride;
    for (int p = a.patch_ptr[s] + lane; p < a.patch_ptr[s + 1]; p += 64) {
      const DPatch P = a.patches[p];
      double sm[13];
      #pragma unroll
      for (int q = 0; q < 13; ++q) sm[q] = 0.0;
      for (int t = P.task_begin; t < P.task_end; ++t)
        #pragma unroll
        for (int q = 0; q < 13; ++q) sm[q] += slots[(int64_t)t * kSlots + q];
      local += sm[S_T] + a.pix_const[2 * p];
      own += sm[S_T_OWN] + a.pix_const[2 * p + 1];
      if (!a.want_grad) continue;
      const cel_image& im = a.images[P.img];
      double L[2], M[2], var[2];
      #pragma unroll
      for (int i = 0; i < 2; ++i) {
        double m = th[3 + i];
        var[i] = exp(th[5 + i]);
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double W = c_W[im.band][c];
          m += W * th[7 + 4 * i + c];
          var[i] += W * W * exp(th[15 + 4 * i + c]);
        }
        L[i] = im.iota * exp(m + 0.5 * var[i]);
        M[i] = im.iota * im.iota * exp(2.0 * m + 2.0 * var[i]);
      }
      // E_s = w0 L0 f0 + w1 L1 f1,  V_s = w0 M0 f0^2 + w1 M1 f1^2 - E_s^2
      const double A0 = sm[S_CE_F0], A1 = sm[S_CE_F1], B00 = sm[S_CV_F00], B11 = sm[S_CV_F11], B01 = sm[S_CV_F01];
      const double gL0 = w0 * A0 - 2.0 * w0 * (w0 * L[0] * B00 + w1 * L[1] * B01);
      const double gL1 = w1 * A1 - 2.0 * w1 * (w0 * L[0] * B01 + w1 * L[1] * B11);
      const double gM0 = w0 * B00, gM1 = w1 * B11;
      const double ga = L[1] * A1 - L[0] * A0 + M[1] * B11 - M[0] * B00 -
                        2.0 * (w0 * L[0] * L[1] * B01 - w0 * L[0] * L[0] * B00 + w1 * L[1] * L[1] * B11 -
                               w1 * L[0] * L[1] * B01);
      g[2] += ga * aa * (1.0 - aa);
      const double gL[2] = {gL0, gL1}, gM[2] = {gM0, gM1};
      #pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double gm = gL[i] * L[i] + 2.0 * gM[i] * M[i];
        const double gv = 0.5 * gL[i] * L[i] + 2.0 * gM[i] * M[i];
        g[3 + i] += gm;
        g[5 + i] += gv * exp(th[5 + i]);
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double W = c_W[im.band][c];
          g[7 + 4 * i + c] += gm * W;
          g[15 + 4 * i + c] += gv * W * W * exp(th[15 + 4 * i + c]);
        }
      }
      // centre: mu = A u + b
      g[0] += im.A[0][0] * sm[S_MU_X] + im.A[1][0] * sm[S_MU_Y];
      g[1] += im.A[0][1] * sm[S_MU_X] + im.A[1][1] * sm[S_MU_Y];
      // covariance: S = A Sigma A^T;  d/dSigma (matrix) = A^T G A
      const double Gxx = sm[S_S_XX], Gxy = 0.5 * sm[S_S_XY], Gyy = sm[S_S_YY];
      const double a00 = im.A[0][0], a01 = im.A[0][1], a10 = im.A[1][0], a11 = im.A[1][1];
      const double h00 = a00 * (Gxx * a00 + Gxy * a10) + a10 * (Gxy * a00 + Gyy * a10);
      const double h01 = a00 * (Gxx * a01 + Gxy * a11) + a10 * (Gxy * a01 + Gyy * a11);
      const double h11 = a01 * (Gxx * a01 + Gxy * a11) + a11 * (Gxy * a01 + Gyy * a11);
      gS[0] += h00;
      gS[1] += 2.0 * h01;
      gS[2] += h11;
      gpi += sm[S_PI];
    }
    // combine the lanes' partial sums (fixed order: deterministic), all of them together; the
    // lane holding a sum puts it in LDS, from where every lane reads them all
    if (a.want_grad) {
      double v[kRed];
      v[0] = local;
      v[1] = own;
      #pragma unroll
      for (int k = 0; k < kParamN; ++k) v[2 + k] = g[k];
      #pragma unroll
      for (int k = 0; k < 3; ++k) v[2 + kParamN + k] = gS[k];
      v[kRed - 1] = gpi;
      const double sv = wave_sums<kRed>(v, lane);
      const int sl = wave_sums_slot<kRed>(lane);
      if (sl >= 0) red[sl] = sv;
    } else {
      const double v[2] = {local, own};
      const double sv = wave_sums<2>(v, lane);
      const int sl = wave_sums_slot<2>(lane);
      if (sl >= 0) red[sl] = sv;
    }
  }
  __syncthreads();
  if (kl_wave) return;
  if (!split) {
    double gk[kThetaN];
    #pragma unroll
    for (int k = 0; k < kThetaN; ++k) gk[k] = 0.0;
    kl_to_lds(gk);
    __syncthreads();
  }
  local = red[0];
  own = red[1];
  if (a.want_grad) {
    #pragma unroll
    for (int k = 0; k < kParamN; ++k) g[k] = red[2 + k];
    #pragma unroll
    for (int k = 0; k < 3; ++k) gS[k] = red[2 + kParamN + k];
    gpi = red[kRed - 1];
  }
  if (lane != 0) return;
  const double kl = klg[0];
  local -= kl;
  own -= kl;
  if (a.want_grad) {
    #pragma unroll
    for (int k = 0; k < kParamN; ++k) g[k] += klg[1 + k];
    // Sigma(angle, radius, axis) chain rule
    const double c = cos(ang), sn = sin(ang), r2 = rad * rad, a2 = axis * axis;
    const double dxx_dt = 2.0 * r2 * c * sn * (a2 - 1.0), dyy_dt = -dxx_dt;
    const double dxy_dt = r2 * (a2 - 1.0) * (c * c - sn * sn);
    g[23] += gS[0] * dxx_dt + gS[1] * dxy_dt + gS[2] * dyy_dt;
    g[24] += 2.0 * (gS[0] * sig[0] + gS[1] * sig[1] + gS[2] * sig[2]);   // d/dlog r
    const double dxx_da = 2.0 * axis * r2 * sn * sn, dyy_da = 2.0 * axis * r2 * c * c,
                 dxy_da = 2.0 * axis * r2 * c * sn;
    g[26] += (gS[0] * dxx_da + gS[1] * dxy_da + gS[2] * dyy_da) * axis * (1.0 - axis);
    g[25] += gpi * prof * (1.0 - prof);
  }
  const int64_t out = (int64_t)vv * a.out_variant_stride + s;
  if (a.err && !isfinite(local)) atomicOr(a.err, CEL_DEVERR_NONFINITE_OBJECTIVE);
  if (a.local) a.local[out] = local;
  if (a.own) a.own[out] = own;
  if (a.want_grad && a.grad) {
    #pragma unroll
    for (int k = 0; k < kParamN; ++k) a.grad[out * kThetaN + k] = g[k];
    #pragma unroll
    for (int k = kParamN; k < kThetaN; ++k) a.grad[out * kThetaN + k] = 0.0;
  }
}

// deterministic sum of n values (fixed per-thread stride order, then a fixed tree)
__global__ __launch_bounds__(256) void k_total(const double* __restrict__ own, int n, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += own[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ----------------------------------------------------------------------------------------
// preparation kernels: per-pixel (count, sky) and per-patch data constants

__global__ __launch_bounds__(256) void k_pixels(const DPatch* __restrict__ patches, const cel_image* __restrict__ images,
                                                const double* __restrict__ knots, const float* __restrict__ pixels,
                                                const int64_t* __restrict__ user_off, float2* __restrict__ xs,
                                                double2* __restrict__ xs64) {
  const DPatch P = patches[blockIdx.x];
  const cel_image& im = images[P.img];
  const double* kn = knots + im.sky_off;
  const int n = P.w * P.h;
  // patch-local coordinates of this thread's pixels, advanced by 256 pixels per pass
  const int step_rows = 256 / P.w, step_cols = 256 - step_rows * P.w;
  int prow = (int)threadIdx.x / P.w, pcol = (int)threadIdx.x - prow * P.w;
  for (int i = threadIdx.x; i < n; i += 256) {
    const int row = P.y0 + prow, col = P.x0 + pcol;
    pcol += step_cols;
    prow += step_rows;
    if (pcol >= P.w) {
      pcol -= P.w;
      prow += 1;
    }
    // bilinear interpolation on a knot grid spanning the image corners (Section 2.2.1)
    double fy = 0, fx = 0;
    int iy = 0, ix = 0;
    if (im.sky_qh > 1) {
      fy = (double)row * (im.sky_qh - 1) / (double)(im.H - 1);
      iy = min(max((int)floor(fy), 0), im.sky_qh - 2);
      fy -= iy;
    }
    if (im.sky_qw > 1) {
      fx = (double)col * (im.sky_qw - 1) / (double)(im.W - 1);
      ix = min(max((int)floor(fx), 0), im.sky_qw - 2);
      fx -= ix;
    }
    const int iy1 = min(iy + 1, im.sky_qh - 1), ix1 = min(ix + 1, im.sky_qw - 1);
    const double sky = (1 - fy) * (1 - fx) * kn[iy * im.sky_qw + ix] + (1 - fy) * fx * kn[iy * im.sky_qw + ix1] +
                       fy * (1 - fx) * kn[iy1 * im.sky_qw + ix] + fy * fx * kn[iy1 * im.sky_qw + ix1];
    const float x = pixels[user_off[blockIdx.x] + i];
    xs[P.off + i] = make_float2(x, (float)sky);
    if (xs64) xs64[P.off + i] = make_double2((double)x, sky);
  }
}

// sum over the patch of C(x) = x log x - x - log x! (all pixels, and owned pixels only)
// data constant of a count: x log x - x - log x! (0 for x = 0)
__device__ __forceinline__ double count_const(double x) { return x > 0 ? x * log(x) - x - lgamma(x + 1.0) : 0.0; }

// the data constants of the counts 0 .. kCountTable - 1
__global__ __launch_bounds__(256) void k_count_table(double* __restrict__ table) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kCountTable) table[i] = count_const((double)i);
}

__global__ __launch_bounds__(256) void k_pixconst(const DPatch* __restrict__ patches, const int32_t* __restrict__ nbr_idx,
                                                  const float2* __restrict__ xs, const double* __restrict__ table,
                                                  double* __restrict__ out, double* __restrict__ sky_min) {
  __shared__ double sh[3][256];
  const DPatch P = patches[blockIdx.x];
  const int n = P.w * P.h;
  double all = 0, own = 0, smin = INFINITY;
  // patch-local coordinates of this thread's pixels, advanced by 256 pixels per pass
  const int step_rows = 256 / P.w, step_cols = 256 - step_rows * P.w;
  int prow = (int)threadIdx.x / P.w, pcol = (int)threadIdx.x - prow * P.w;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float2 v = xs[P.off + i];
    const double x = v.x;
    smin = fmin(smin, (double)v.y);
    // integer counts below the table's size from the table (the same values)
    const double c = (x >= 0 && x < (double)kCountTable && x == floor(x)) ? table[(int)x] : count_const(x);
    all += c;
    const int col = P.x0 + pcol, row = P.y0 + prow;
    pcol += step_cols;
    prow += step_rows;
    if (pcol >= P.w) {
      pcol -= P.w;
      prow += 1;
    }
    bool mine = true;
    for (int nb = P.nbr_begin; nb < P.nbr_end; ++nb) {
      const DPatch Q = patches[nbr_idx[nb]];
      if (Q.src < P.src && col >= Q.x0 && col < Q.x0 + Q.w && row >= Q.y0 && row < Q.y0 + Q.h) mine = false;
    }
    if (mine) own += c;
  }
  sh[0][threadIdx.x] = all;
  sh[1][threadIdx.x] = own;
  sh[2][threadIdx.x] = smin;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
      sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = sh[0][0];
    out[2 * blockIdx.x + 1] = sh[1][0];
    sky_min[blockIdx.x] = sh[2][0];
  }
}

// ----------------------------------------------------------------------------------------
// launch wrappers

template <typename T>
hipError_t launch_prep_tables(const PrepArgs& a, int n_patches_launch, int n_variants, hipStream_t st) {
  if (n_patches_launch <= 0 || n_variants <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_tables<T>, dim3(n_patches_launch, n_variants), dim3(64), 0, st, a);
  return hipGetLastError();
}

template <typename T, int PPL, bool GRAD>
static hipError_t fused_dispatch(const FusedArgs<T>& a, int nexp, int ndev, int n_items, int n_var,
                                 hipStream_t st) {
  dim3 grid(n_items, n_var);
  FusedArgs<T> k = a;
  k.unscale[0] = 1.0 / kExpScale;
  k.unscale[1] = 1.0 / (kExpScale * kExpScale);
  if (nexp == 6 && ndev == 8)
    hipLaunchKernelGGL((k_fused<T, PPL, GRAD, 6, 8>), grid, dim3(64), 0, st, k);
  else
    hipLaunchKernelGGL((k_fused<T, PPL, GRAD, 8, 8>), grid, dim3(64), 0, st, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int nexp, int ndev, int ppl, bool grad, int n_items,
                        int n_variants, hipStream_t st) {
  if (n_items <= 0 || n_variants <= 0) return hipSuccess;
  switch (ppl * 2 + (grad ? 1 : 0)) {
    case 2: return fused_dispatch<T, 1, false>(a, nexp, ndev, n_items, n_variants, st);
    case 3: return fused_dispatch<T, 1, true>(a, nexp, ndev, n_items, n_variants, st);
    case 4: return fused_dispatch<T, 2, false>(a, nexp, ndev, n_items, n_variants, st);
    case 5: return fused_dispatch<T, 2, true>(a, nexp, ndev, n_items, n_variants, st);
    case 8: return fused_dispatch<T, 4, false>(a, nexp, ndev, n_items, n_variants, st);
    case 9: return fused_dispatch<T, 4, true>(a, nexp, ndev, n_items, n_variants, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_maps(const MapArgs& a, int nexp, int ndev, int ppl, int n_items, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const bool std_prof = nexp == 6 && ndev == 8;
  if (ppl == 1) {
    if (std_prof) hipLaunchKernelGGL((k_maps<T, 1, 6, 8>), dim3(n_items), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_maps<T, 1, 8, 8>), dim3(n_items), dim3(64), 0, st, a);
  } else if (ppl == 2) {
    if (std_prof) hipLaunchKernelGGL((k_maps<T, 2, 6, 8>), dim3(n_items), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_maps<T, 2, 8, 8>), dim3(n_items), dim3(64), 0, st, a);
  } else if (ppl == 4) {
    if (std_prof) hipLaunchKernelGGL((k_maps<T, 4, 6, 8>), dim3(n_items), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_maps<T, 4, 8, 8>), dim3(n_items), dim3(64), 0, st, a);
  } else if (ppl == 8) {
    if (std_prof) hipLaunchKernelGGL((k_maps<T, 8, 6, 8>), dim3(n_items), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_maps<T, 8, 8, 8>), dim3(n_items), dim3(64), 0, st, a);
  } else if (ppl == -1) {   // runs along rows, values by recurrence
    if (std_prof) hipLaunchKernelGGL((k_maps_runs<T, 6, 8>), dim3(n_items), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_maps_runs<T, 8, 8>), dim3(n_items), dim3(64), 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, int n_variants, hipStream_t st) {
  if (a.n_jobs <= 0 || n_variants <= 0) return hipSuccess;
  // the KL on its own wavefront while all blocks fit on the chip at once (two-wavefront
  // blocks of k_finalize's ~210 registers per lane: four per compute unit, 256 units)
  constexpr int64_t kSplitMaxBlocks = 1024;
  const bool split = (int64_t)a.n_jobs * n_variants <= kSplitMaxBlocks;
  hipLaunchKernelGGL(k_finalize, dim3(a.n_jobs, n_variants), dim3(split ? 128 : 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_total(const double* own, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_total, dim3(1), dim3(256), 0, st, own, n, out);
  return hipGetLastError();
}

hipError_t launch_pixels(const DPatch* patches, const cel_image* images, const double* knots, const float* pixels,
                         const int64_t* user_off, float2* xs, double2* xs64, int n_patches, hipStream_t st) {
  if (n_patches <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pixels, dim3(n_patches), dim3(256), 0, st, patches, images, knots, pixels, user_off, xs, xs64);
  return hipGetLastError();
}

// Point values z of a source (type, log flux, colours, position, shape) as unconstrained
// parameters whose variational distribution is the point mass at z (Section 3.1 evaluates
// the likelihood at sampled z): the type logit at +/-infinity (q(star) exactly 1 or 0),
// every variance exp(-infinity) = 0, both types' flux and colour means at the point's
// values, the profile and axis logits of the point's weights.  With zero variances the
// delta method's correction vanishes and the objective's pixel terms are the Poisson
// log-likelihood at z.  A row outside the support (profile weight not in [0, 1], axis
// ratio not in (0, 1], or a non-finite value) is marked in ok[] (null: not recorded).
__global__ __launch_bounds__(256) void k_point_theta(const double* __restrict__ z, int64_t n,
                                                     double* __restrict__ theta, uint8_t* __restrict__ ok) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* zi = z + i * CEL_Z_N;
  double* t = theta + i * kThetaN;
  const double inf = __builtin_huge_val();
  bool good = zi[10] >= 0.0 && zi[10] <= 1.0 && zi[11] > 0.0 && zi[11] <= 1.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) good = good && isfinite(zi[k]);
  t[0] = zi[0];
  t[1] = zi[1];
  t[2] = zi[2] != 0.0 ? inf : -inf;
  t[3] = t[4] = zi[3];
  t[5] = t[6] = -inf;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    t[7 + c] = t[11 + c] = zi[4 + c];
    t[15 + c] = t[19 + c] = -inf;
  }
  t[23] = zi[8];
  t[24] = zi[9];
  // logit(p) = log p - log(1 - p): -inf at 0, +inf at 1
  t[25] = log(zi[10]) - log1p(-zi[10]);
  t[26] = log(zi[11]) - log1p(-zi[11]);
#pragma unroll
  for (int k = kParamN; k < kThetaN; ++k) t[k] = 0.0;
  if (ok) ok[i] = good ? 1 : 0;
}

// log-likelihood -infinity for the selected sources' candidates outside the support (ok[] of
// k_point_theta; rows [candidate][source], S sources per candidate)
__global__ __launch_bounds__(256) void k_support(const uint8_t* __restrict__ ok, const uint8_t* __restrict__ mask,
                                                 int S, int64_t n, double* __restrict__ ll) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && mask[i % S] && !ok[i]) ll[i] = -__builtin_huge_val();
}

// log p(w_s | a_s) at point values (the start distribution of the annealed importance
// sampler, Section 3.1), over the point layout's coordinates, from the model's priors
// (Section 2.1): log r normal given the type, the colours from the type's Gaussian
// mixture, and for a galaxy log radius normal, profile weight and axis ratio beta, the angle
// uniform on [0, pi); the position's uniform prior is a constant and left out.  -infinity
// outside the support.  One thread per point.
__global__ __launch_bounds__(256) void k_log_prior(const DPrior* __restrict__ pr, const double* __restrict__ z,
                                                   int64_t n, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const double* zi = z + r * CEL_Z_N;
  bool good = zi[10] >= 0.0 && zi[10] <= 1.0 && zi[11] > 0.0 && zi[11] <= 1.0;
  for (int k = 0; k < 12; ++k) good = good && isfinite(zi[k]);
  if (!good) {
    out[r] = -__builtin_huge_val();
    return;
  }
  const int i = zi[2] != 0.0 ? 1 : 0;
  const double kLogTwoPi = 1.8378770664093454836;
  auto normal = [&](double x, double mean, double var) {
    const double d = x - mean;
    return -0.5 * (kLogTwoPi + log(var)) - 0.5 * d * d / var;
  };
  double lp = normal(zi[3], pr->r[i][0], pr->r[i][1]);
  // colour mixture: log sum_j w_j N(c; m_j, C_j), largest term factored out
  double t[CEL_N_COLOUR_COMPONENTS], tmax = -__builtin_huge_val();
  for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) {
    double maha = 0.0;
    double d[4];
    for (int a = 0; a < 4; ++a) d[a] = zi[4 + a] - pr->c_mean[i][j][a];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) maha += d[a] * pr->c_prec[i][j][a][b] * d[b];
    const bool used = pr->c_logw[i][j] > -1e299;
    t[j] = used ? pr->c_logw[i][j] - 2.0 * kLogTwoPi - 0.5 * pr->c_logdet[i][j] - 0.5 * maha : -__builtin_huge_val();
    tmax = fmax(tmax, t[j]);
  }
  double sum = 0.0;
  for (int j = 0; j < CEL_N_COLOUR_COMPONENTS; ++j) sum += exp(t[j] - tmax);
  lp += tmax + log(sum);
  if (i == 0) {
    const double pa = pr->profile[0], pb = pr->profile[1], aa = pr->axis[0], ab = pr->axis[1];
    lp += normal(zi[9], pr->radius[0], pr->radius[1]);
    lp += (pa - 1.0) * log(zi[10]) + (pb - 1.0) * log1p(-zi[10]) - pr->lbeta_profile;
    lp += (aa - 1.0) * log(zi[11]) + (ab - 1.0) * log1p(-zi[11]) - pr->lbeta_axis;
    lp -= 1.1447298858494001741;   // log(pi): the angle's uniform density on [0, pi)
  }
  out[r] = lp;
}

hipError_t launch_log_prior(const DPrior* prior, const double* z, int64_t n, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_log_prior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, prior, z, n, out);
  return hipGetLastError();
}

hipError_t launch_point_theta(const double* z, int64_t n, double* theta, uint8_t* ok, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_point_theta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, z, n, theta, ok);
  return hipGetLastError();
}

hipError_t launch_support_masked(const uint8_t* ok, const uint8_t* mask, int S, int64_t n, double* ll, hipStream_t st) {
  if (n <= 0 || S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_support, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ok, mask, S, n, ll);
  return hipGetLastError();
}

hipError_t launch_count_table(double* table, hipStream_t st) {
  hipLaunchKernelGGL(k_count_table, dim3((kCountTable + 255) / 256), dim3(256), 0, st, table);
  return hipGetLastError();
}

hipError_t launch_pixconst(const DPatch* patches, const int32_t* nbr_idx, const float2* xs, const double* table,
                           double* out, double* sky_min, int n_patches, hipStream_t st) {
  if (n_patches <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pixconst, dim3(n_patches), dim3(256), 0, st, patches, nbr_idx, xs, table, out, sky_min);
  return hipGetLastError();
}

template hipError_t launch_prep_tables<float>(const PrepArgs&, int, int, hipStream_t);
template hipError_t launch_prep_tables<double>(const PrepArgs&, int, int, hipStream_t);
template hipError_t launch_maps<float>(const MapArgs&, int, int, int, int, hipStream_t);
template hipError_t launch_maps<double>(const MapArgs&, int, int, int, int, hipStream_t);
template hipError_t launch_fused<float>(const FusedArgs<float>&, int, int, int, bool, int, int,
                                        hipStream_t);
template hipError_t launch_fused<double>(const FusedArgs<double>&, int, int, int, bool, int, int,
                                         hipStream_t);

}  // namespace celmi
