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

#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "pixmath.h"
#include "plan.h"

namespace celmi {

constexpr int kN = kParamN;   // 27
static_assert(((kN + 1) / 2) % 2 == 0, "the Jacobi half-columns hold an even number of rows");
constexpr int kLd = kN + 1;   // padded LDS row



// Hessian of KL_s in the unconstrained coordinates (the same KL as the objective: the type
// KL, the normal KL of log r, the colour bound F = -log sum_j w_j exp(-D_j), and minus the
// log prior densities of the radius, profile and axis point masses), times sc, added into
// B (27 rows of stride LD).  KL = KL_a(eta) + KL_radius + KL_profile + KL_axis
// + (1 - a) K_0 + a K_1; grad F = sum_j xi_j dD_j and
// hess F = sum_j xi_j (d2D_j - dD_j dD_j^T) + grad F grad F^T in the 8 colour variables.
// Computed by a whole wavefront (all 64 lanes active, B in LDS): lane
// 8 i + j takes prior colour component j of type i -- its weight xi_j, dD_j and d2D_j --
// and the sums over j of xi_j (d2D_j - dD_j dD_j^T) and xi_j dD_j are formed through LDS
// in fixed order (work: 16 x 44 and 2 x 44 doubles); lanes then add the two 8 x 8 colour
// blocks and lane 0 the remaining terms.  Ends after a barrier.
constexpr int kKlw = 44;   // 36 upper-triangle entries of the 8 x 8 block + 8 gradient entries
template <int LD>
__device__ void kl_hessian_wave(const DPrior& pr, const double* th, double (*B)[LD], double sc, int lane,
                                double (*work)[kKlw], double (*sums)[kKlw]) {
  static_assert(CEL_N_COLOUR_COMPONENTS == 8, "one lane per prior colour component, groups of 8");
  const int i = (lane >> 3) & 1, j = lane & 7;
  double cm[4], cv[4], lcv = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {   // selects, not a lane-dependent index into th
    cm[k] = i ? th[11 + k] : th[7 + k];
    const double l = i ? th[19 + k] : th[15 + k];
    cv[k] = exp(l);
    lcv += l;
  }
  double tr = 0, maha = 0, dD[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    tr += pr.c_prec[i][j][k][k] * cv[k];
    double r = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) r += pr.c_prec[i][j][k][l] * (cm[l] - pr.c_mean[i][j][l]);
    dD[k] = r;
    dD[4 + k] = 0.5 * (pr.c_prec[i][j][k][k] * cv[k] - 1.0);
    maha += (cm[k] - pr.c_mean[i][j][k]) * r;
  }
  const double e = pr.c_logw[i][j] - 0.5 * (tr + maha - 4.0 + pr.c_logdet[i][j] - lcv);
  double mx = e;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const double ex = exp(e - mx);
  double z = ex;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) z += __shfl_xor(z, off, 64);
  const double xi = ex / z;
  const double kc = -(mx + log(z));   // the colour bound of type i
  if (lane < 16) {
    int n = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int w = u; w < 8; ++w) {
        double d2 = 0.0;
        if (u < 4 && w < 4) d2 = pr.c_prec[i][j][u][w];
        else if (u == w) d2 = 0.5 * pr.c_prec[i][j][u - 4][u - 4] * cv[u - 4];
        work[lane][n++] = xi * (d2 - dD[u] * dD[w]);
      }
#pragma unroll
    for (int u = 0; u < 8; ++u) work[lane][36 + u] = xi * dD[u];
  }
  __syncthreads();
  for (int e2 = lane; e2 < 2 * kKlw; e2 += 64) {
    const int ii = e2 / kKlw, q = e2 % kKlw;
    double acc = 0;
    for (int jj = 0; jj < 8; ++jj) acc += work[8 * ii + jj][q];
    sums[ii][q] = acc;
  }
  __syncthreads();
  const double eta = th[2], a = sigmoid(eta), aa = a * (1.0 - a);
  // colour blocks: entry (u, w) of type ii, lanes 0..63 twice
  for (int e2 = lane; e2 < 2 * 64; e2 += 64) {
    const int ii = e2 / 64, u = (e2 % 64) / 8, w = e2 % 8;
    const int lo = u < w ? u : w, hi = u < w ? w : u;
    const int n = lo * 8 - lo * (lo - 1) / 2 + (hi - lo);
    const double q = ii == 0 ? 1.0 - a : a;
    const double hf = sums[ii][n] + sums[ii][36 + u] * sums[ii][36 + w];
    const int iu = u < 4 ? 7 + 4 * ii + u : 15 + 4 * ii + (u - 4);
    const int iw = w < 4 ? 7 + 4 * ii + w : 15 + 4 * ii + (w - 4);
    B[iu][iw] += sc * (q * hf);
  }
  const double kc1 = __shfl(kc, 8, 64);
  if (lane == 0) {
    double K[2];
    const double kcs[2] = {kc, kc1};
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const double rm = th[3 + ii], lrv = th[5 + ii], rv = exp(lrv);
      const double R1 = pr.r[ii][0], R2 = pr.r[ii][1];
      const double q = ii == 0 ? 1.0 - a : a;
      const double sg = ii == 0 ? -aa : aa;   // d^2 KL / d eta d theta_k = sg dK_i/dtheta_k
      K[ii] = 0.5 * (log(R2) - lrv) + (rv + (rm - R1) * (rm - R1)) / (2.0 * R2) - 0.5 + kcs[ii];
      const double dm = (rm - R1) / R2, dv = -0.5 + rv / (2.0 * R2);
      B[3 + ii][3 + ii] += sc * (q / R2);
      B[5 + ii][5 + ii] += sc * (q * rv / (2.0 * R2));
      B[2][3 + ii] += sc * (sg * dm);
      B[3 + ii][2] += sc * (sg * dm);
      B[2][5 + ii] += sc * (sg * dv);
      B[5 + ii][2] += sc * (sg * dv);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int iu = u < 4 ? 7 + 4 * ii + u : 15 + 4 * ii + (u - 4);
        B[2][iu] += sc * (sg * sums[ii][36 + u]);
        B[iu][2] += sc * (sg * sums[ii][36 + u]);
      }
    }
    // type weight: dKL/deta = a(1-a) [eta - logit A + K1 - K0]
    const double t = eta - pr.logit_a + K[1] - K[0];
    B[2][2] += sc * (aa * (1.0 - 2.0 * a) * t + aa);
    // point masses
    B[24][24] += sc * (1.0 / pr.radius[1]);
    {
      const double p = sigmoid(th[25]);
      B[25][25] += sc * ((pr.profile[0] + pr.profile[1] - 2.0) * p * (1.0 - p));
    }
    {
      const double p = sigmoid(th[26]);
      B[26][26] += sc * ((pr.axis[0] + pr.axis[1] - 2.0) * p * (1.0 - p));
    }
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------------------
// Analytic Hessian of the pixel part of L_s (Section 4.3 uses a dense Newton Hessian).
//
// Per patch the pixel sum depends on theta_s through 11 primitives
//   y = (a, L0, L1, e0, e1, mu_x, mu_y, S_xx, S_xy, S_yy, pi)
// (type probability, flux moments L_i = E[l | a=i] and e_i = expm1(Var log l | a=i), the
// pixel-frame centre and galaxy covariance, the de Vaucouleurs weight), with
//   E_s = w0 L0 f0 + w1 L1 f1,  V_s = w0 L0^2 e0 f0^2 + w1 L1^2 e1 f1^2 + w0 w1 d^2,
//   d = L0 f0 - L1 f1,  w0 = 1 - a, w1 = a.
// For T(E, V) = -E + x (log E - V / (2 E^2)):  T_E = c_E, T_V = c_V,
//   T_EE = -x/E^2 - 3 x V / E^4, T_EV = x / E^3, T_VV = 0, so per pixel
//   d2T/du dv = T_EE E_u E_v + T_EV (E_u V_v + E_v V_u) + c_E E_uv + c_V V_uv.
// f0, f1 and their first and second derivatives in (mu, S, pi) come from the Gaussian
// identities (N = normal density with precision P, u = P (p - m)):
//   dN/dmu = N u,  d2N/dmu dmu = N (u u^T - P),  dN/dC[dC] = N (u^T dC u - tr(P dC)) / 2,
//   d2N/dmu dC[dC] = dN[dC] u - N P dC u,
//   d2N/dC dC[dC1, dC2] = dN[dC1] dN[dC2] / N - N u^T dC1 P dC2 u + N tr(dC1 P dC2 P) / 2,
// with dC = tau dS for a galaxy component.  The kernel sums G_u and the 66 entries Q_uv
// per work item; k_hess_finalize maps them to theta_s by the chain rule.

constexpr int kPrim = 11;
constexpr int kHQ = 66;
constexpr int kHSlots = 80;   // T, T_own, G[11], Q[66], pad

__host__ __device__ constexpr int qidx(int u, int v) { return u * kPrim - u * (u - 1) / 2 + (v - u); }
__host__ __device__ constexpr int zidx(int i, int j) { return i * 6 - i * (i - 1) / 2 + (j - i); }

template <typename T>
struct PixH {
  T f0, f1;
  T g0[6];   // mu_x, mu_y, S_xx, S_xy, S_yy, pi
  T g1[2];
  T h0[21];  // upper triangle (zidx)
  T h1[3];   // xx, xy, yy
};

// one galaxy component of one profile: value, first derivatives (per profile) and the
// profile-weighted second derivatives in (mu, S)
template <typename T>
__device__ __forceinline__ void gal_hess(const T* q, T Pxx, T Pxy, T Pyy, T lw, const T* gt, T wP, T dx, T dy, T xx,
                                         T xy, T yy, T& f, T* gm, T* gs, T* hmm, T* hms, T* hss) {
  const T ux = fma(Pxx, dx, Pxy * dy);
  const T uy = fma(Pxy, dx, Pyy * dy);
  const T N = comp_value<T>(q, xx, xy, yy);
  const T qxx = fma(ux, ux, -Pxx), qxy = fma(ux, uy, -Pxy), qyy = fma(uy, uy, -Pyy);
  const T tau = gt[0], tau2 = gt[1];
  const T Nh = (T)0.5 * tau * N;
  f += N;
  gm[0] = fma(N, ux, gm[0]);
  gm[1] = fma(N, uy, gm[1]);
  const T Nxx = Nh * qxx, Nxy = (T)2 * Nh * qxy, Nyy = Nh * qyy;
  gs[0] += Nxx;
  gs[1] += Nxy;
  gs[2] += Nyy;
  const T Nw = N * wP;
  hmm[0] = fma(Nw, qxx, hmm[0]);
  hmm[1] = fma(Nw, qxy, hmm[1]);
  hmm[2] = fma(Nw, qyy, hmm[2]);
  const T Ntw = Nw * tau;
  const T vxx_x = ux * Pxx, vxx_y = ux * Pxy;
  const T vxy_x = fma(Pxx, uy, Pxy * ux), vxy_y = fma(Pxy, uy, Pyy * ux);
  const T vyy_x = uy * Pxy, vyy_y = uy * Pyy;
  const T w0e = Nxx * wP, w1e = Nxy * wP, w2e = Nyy * wP;
  // each term is one fma into the entry's accumulator (the sign of the terms in N P rides on
  // the operand)
  hms[0] = fma(w0e, ux, hms[0]);
  hms[3] = fma(w0e, uy, hms[3]);
  hms[1] = fma(w1e, ux, hms[1]);
  hms[4] = fma(w1e, uy, hms[4]);
  hms[2] = fma(w2e, ux, hms[2]);
  hms[5] = fma(w2e, uy, hms[5]);
  hms[0] = fma(-Ntw, vxx_x, hms[0]);
  hms[3] = fma(-Ntw, vxx_y, hms[3]);
  hms[1] = fma(-Ntw, vxy_x, hms[1]);
  hms[4] = fma(-Ntw, vxy_y, hms[4]);
  hms[2] = fma(-Ntw, vyy_x, hms[2]);
  hms[5] = fma(-Ntw, vyy_y, hms[5]);
  const T q1 = (T)2 * qxy;
  const T Nwt2 = Nw * tau2;
  hss[0] = fma(Nwt2, (T)0.25 * qxx * qxx - ux * vxx_x, hss[0]);
  hss[1] = fma(Nwt2, (T)0.25 * qxx * q1 - ux * vxy_x, hss[1]);
  hss[2] = fma(Nwt2, (T)0.25 * qxx * qyy - ux * vyy_x, hss[2]);
  hss[3] = fma(Nwt2, (T)0.25 * q1 * q1 - fma(uy, vxy_x, ux * vxy_y), hss[3]);
  hss[4] = fma(Nwt2, (T)0.25 * q1 * qyy - uy * vxy_y, hss[4]);
  hss[5] = fma(Nwt2, (T)0.25 * qyy * qyy - uy * vyy_y, hss[5]);
#pragma unroll
  for (int e = 0; e < 6; ++e) hss[e] = fma(Nw, gt[2 + e], hss[e]);
}

template <typename T, int NEXP, int NDEV>
__device__ __forceinline__ void eval_own_hess(const Table<T>* __restrict__ tb, int K, T px, T py, const T* box,
                                              PixH<T>& o) {
  T fe = 0, fd = 0, gme[2] = {0, 0}, gmd[2] = {0, 0}, gse[3] = {0, 0, 0}, gsd[3] = {0, 0, 0};
  T hmm[3] = {0, 0, 0}, hms[6] = {0, 0, 0, 0, 0, 0}, hss[6] = {0, 0, 0, 0, 0, 0};
  T f1 = 0, g1x = 0, g1y = 0, h1[3] = {0, 0, 0};
  const T pi = tb->hdr[7], omp = (T)1 - pi;
  __builtin_assume(K >= 1);   // images have 1..kMaxPsf PSF components (checked at prepare)
  for (int k = 0; k < K; ++k) {
    const T mx = tb->star[k][0], my = tb->star[k][1];
    const T dx = px - mx, dy = py - my;
    const T xx = dx * dx, xy = (T)2 * dx * dy, yy = dy * dy;
    const auto d2k = uniform_cut_key(box_dist2<T>(mx, my, box));
    // the cut radii of this PSF component, read before any is used (one wait for all)
    T rc[NEXP + NDEV];
#pragma unroll
    for (int j = 0; j < NEXP + NDEV; ++j) rc[j] = tb->rc2[k][j < NEXP ? j : kMaxProf + (j - NEXP)];
    if (!(d2k > cut_key(tb->rc2s[k]))) {
      const T Pxx = tb->star[k][2], Pxy = tb->star[k][3], Pyy = tb->star[k][4];
      const T ux = fma(Pxx, dx, Pxy * dy), uy = fma(Pxy, dx, Pyy * dy);
      const T N = comp_value<T>(tb->sq[k], xx, xy, yy);
      f1 += N;
      g1x = fma(N, ux, g1x);
      g1y = fma(N, uy, g1y);
      h1[0] = fma(N, fma(ux, ux, -Pxx), h1[0]);
      h1[1] = fma(N, fma(ux, uy, -Pxy), h1[1]);
      h1[2] = fma(N, fma(uy, uy, -Pyy), h1[2]);
    }
#pragma unroll
    for (int j = 0; j < NEXP; ++j)
      if (!(d2k > cut_key(rc[j])))
        gal_hess<T>(tb->gq[k][j], tb->gal[k][j][0], tb->gal[k][j][1], tb->gal[k][j][2], tb->gal[k][j][3],
                    tb->gt[k][j], omp, dx, dy, xx, xy, yy, fe, gme, gse, hmm, hms, hss);
#pragma unroll
    for (int j = 0; j < NDEV; ++j)
      if (!(d2k > cut_key(rc[NEXP + j])))
        gal_hess<T>(tb->gq[k][kMaxProf + j], tb->gal[k][kMaxProf + j][0], tb->gal[k][kMaxProf + j][1],
                    tb->gal[k][kMaxProf + j][2], tb->gal[k][kMaxProf + j][3], tb->gt[k][kMaxProf + j], pi, dx, dy, xx,
                    xy, yy, fd, gmd, gsd, hmm, hms, hss);
  }
  o.f1 = f1;
  o.g1[0] = g1x;
  o.g1[1] = g1y;
  o.h1[0] = h1[0];
  o.h1[1] = h1[1];
  o.h1[2] = h1[2];
  o.f0 = fma(pi, fd, omp * fe);
  o.g0[0] = fma(pi, gmd[0], omp * gme[0]);
  o.g0[1] = fma(pi, gmd[1], omp * gme[1]);
#pragma unroll
  for (int e = 0; e < 3; ++e) o.g0[2 + e] = fma(pi, gsd[e], omp * gse[e]);
  o.g0[5] = fd - fe;
  o.h0[zidx(0, 0)] = hmm[0];
  o.h0[zidx(0, 1)] = hmm[1];
  o.h0[zidx(1, 1)] = hmm[2];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    o.h0[zidx(0, 2 + e)] = hms[e];
    o.h0[zidx(1, 2 + e)] = hms[3 + e];
  }
  o.h0[zidx(2, 2)] = hss[0];
  o.h0[zidx(2, 3)] = hss[1];
  o.h0[zidx(2, 4)] = hss[2];
  o.h0[zidx(3, 3)] = hss[3];
  o.h0[zidx(3, 4)] = hss[4];
  o.h0[zidx(4, 4)] = hss[5];
  o.h0[zidx(0, 5)] = gmd[0] - gme[0];
  o.h0[zidx(1, 5)] = gmd[1] - gme[1];
#pragma unroll
  for (int e = 0; e < 3; ++e) o.h0[zidx(2 + e, 5)] = gsd[e] - gse[e];
  o.h0[zidx(5, 5)] = 0;
}

struct HessArgs {
  const DTask* tasks;
  const int32_t* order;
  const DPatch* patches;
  const int32_t* nbr_idx;
  const void* tables;          // variant-0 tables
  const void* xs;
  const void* maps;
  double* hslots;              // [n_tasks][kHSlots]
  const uint8_t* active;
  const int32_t* img_npsf;
};

// The float form is held to at most 168 VGPRs, three wavefronts per SIMD (its live set fits
// there without spilling; at the two wavefronts that 194 VGPRs allowed the kernel stalled on
// latency).  The double form keeps its natural allocation.
template <typename T, int NEXP, int NDEV>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_hess(HessArgs a) {
  const int pos = xcd_position((int)blockIdx.x, (int)gridDim.x);
  const int t = a.order ? a.order[pos] : pos;
  const DTask task = a.tasks[t];
  const DPatch P = a.patches[task.patch];
  if (a.active && !a.active[P.src]) return;
  const Table<T>* __restrict__ tb = reinterpret_cast<const Table<T>*>(a.tables) + task.patch;
  const int K = a.img_npsf[P.img];
  const int lane = threadIdx.x;
  const T L0 = tb->hdr[0], L1 = tb->hdr[1], w0 = tb->hdr[2], w1 = tb->hdr[3];
  const T e0 = tb->hdr[8], e1 = tb->hdr[9];
  const T w01 = w0 * w1, aa = w1, oma2 = (T)1 - (T)2 * aa;
  double tsum = 0, town = 0;
  T G[kPrim], Q[kHQ];
#pragma unroll
  for (int u = 0; u < kPrim; ++u) G[u] = 0;
#pragma unroll
  for (int u = 0; u < kHQ; ++u) Q[u] = 0;
  // this lane's patch-local pixel coordinates, advanced by 64 pixels per pass with a carry
  const int step_rows = 64 / P.w, step_cols = 64 - step_rows * P.w;
  int row = (task.pix_begin + lane) / P.w;
  int col = task.pix_begin + lane - row * P.w;
  for (int base = task.pix_begin; base < task.pix_end; base += 64) {
    int idx = base + lane;
    const bool valid = idx < task.pix_end;
    if (!valid) idx = task.pix_begin;
    T xv, sky;
    if constexpr (sizeof(T) == 8) {
      const double2 xs = reinterpret_cast<const double2*>(a.xs)[P.off + idx];
      xv = xs.x; sky = xs.y;
    } else {
      const float2 xs = reinterpret_cast<const float2*>(a.xs)[P.off + idx];
      xv = xs.x; sky = xs.y;
    }
    int ibox[4];
    run_box<int>(base, min(base + 64, task.pix_end), P.w, ibox);
    const T box[4] = {(T)ibox[0], (T)ibox[1], (T)ibox[2], (T)ibox[3]};
    PixH<T> o;
    eval_own_hess<T, NEXP, NDEV>(tb, K, (T)col, (T)row, box, o);
    T Eb = sky, Vb = 0;
    bool own = true;
    for (int nb = P.nbr_begin; nb < P.nbr_end; ++nb) {
      const DPatch Qp = a.patches[a.nbr_idx[nb]];
      const int ox = P.x0 - Qp.x0, oy = P.y0 - Qp.y0;
      // a neighbour whose rectangle misses this pass's pixel box is skipped as a whole
      if (ibox[0] + ox >= Qp.w || ibox[1] + ox < 0 || ibox[2] + oy >= Qp.h || ibox[3] + oy < 0) continue;
      const int cx = col + ox, cy = row + oy;
      if (valid && (unsigned)cx < (unsigned)Qp.w && (unsigned)cy < (unsigned)Qp.h) {
        const int64_t at = Qp.off + (cy * Qp.w + cx);
        if constexpr (sizeof(T) == 8) {
          const double2 ev = reinterpret_cast<const double2*>(a.maps)[at];
          Eb += ev.x; Vb += ev.y;
        } else {
          const float2 ev = reinterpret_cast<const float2*>(a.maps)[at];
          Eb += ev.x; Vb += ev.y;
        }
        if (Qp.src < P.src) own = false;
      }
    }
    const T f0 = o.f0, f1 = o.f1;
    const T d = L0 * f0 - L1 * f1;
    const T Es = w0 * L0 * f0 + w1 * L1 * f1;
    const T k0 = w0 * L0 * L0 * e0, k1 = w1 * L1 * L1 * e1;
    const T Vs = fma(k0 * f0, f0, fma(k1 * f1, f1, w01 * d * d));
    const T E = Eb + Es, V = Vb + Vs, x = xv;
    const T invE = frcp<T>(E);
    const T xr = x * invE * invE;
    T Tm = (x > (T)0 ? x_log_ratio<T>(x, E) : (T)0) - (E - x) - (T)0.5 * xr * V;
    T cE = fma(xr * invE, V, (x - E) * invE);
    T cV = (T)-0.5 * xr;
    T TEE = -xr - (T)3 * xr * V * invE * invE;
    T TEV = xr * invE;
    if (!valid) Tm = cE = cV = TEE = TEV = 0;
    tsum += (double)Tm;
    town += own ? (double)Tm : 0.0;
    // z-derivatives of f1 (zero outside mu) and of d
    T g1z[6], dz[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      g1z[j] = j < 2 ? o.g1[j] : (T)0;
      dz[j] = L0 * o.g0[j] - L1 * g1z[j];
    }
    // the (z, z) block: with E_zz = w0 L0 h0 + w1 L1 h1 and
    //   V_zz = 2 (k0 (g0 g0^T + f0 h0) + k1 (g1 g1^T + f1 h1) + w01 (dz dz^T + d (L0 h0 - L1 h1))),
    // c_E E_zz + c_V V_zz = rho0 h0 + rho1 h1 + 2 c_V (k0 g0 g0^T + k1 g1 g1^T + w01 dz dz^T),
    // rho0 = c_E w0 L0 + 2 c_V (k0 f0 + w01 L0 d), rho1 = c_E w1 L1 + 2 c_V (k1 f1 - w01 L1 d)
    // (g1 and h1 vanish outside the centre coordinates z < 2)
    const T cV2 = (T)2 * cV;
    const T rho0 = fma(cE, w0 * L0, cV2 * fma(k0, f0, w01 * L0 * d));
    const T rho1 = fma(cE, w1 * L1, cV2 * fma(k1, f1, -w01 * L1 * d));
    T ag[6], cd[6], bg[2];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      ag[j] = cV2 * k0 * o.g0[j];
      cd[j] = cV2 * w01 * dz[j];
    }
    bg[0] = cV2 * k1 * g1z[0];
    bg[1] = cV2 * k1 * g1z[1];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
      for (int j = i; j < 6; ++j) {
        T q = Q[qidx(5 + i, 5 + j)];
        q = fma(rho0, o.h0[zidx(i, j)], q);
        if (i < 2 && j < 2) {
          q = fma(rho1, o.h1[i + j], q);
          q = fma(bg[i], g1z[j], q);
        }
        q = fma(ag[i], o.g0[j], q);
        q = fma(cd[i], dz[j], q);
        Q[qidx(5 + i, 5 + j)] = q;
      }
    }
    T Eu[kPrim], Vu[kPrim];
    Eu[0] = -d;
    Eu[1] = w0 * f0;
    Eu[2] = w1 * f1;
    Eu[3] = 0;
    Eu[4] = 0;
    Vu[0] = -L0 * L0 * e0 * f0 * f0 + L1 * L1 * e1 * f1 * f1 + oma2 * d * d;
    Vu[1] = (T)2 * w0 * L0 * e0 * f0 * f0 + (T)2 * w01 * d * f0;
    Vu[2] = (T)2 * w1 * L1 * e1 * f1 * f1 - (T)2 * w01 * d * f1;
    Vu[3] = w0 * L0 * L0 * f0 * f0;
    Vu[4] = w1 * L1 * L1 * f1 * f1;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      Eu[5 + j] = w0 * L0 * o.g0[j] + w1 * L1 * g1z[j];
      Vu[5 + j] = (T)2 * (k0 * f0 * o.g0[j] + k1 * f1 * g1z[j] + w01 * d * dz[j]);
    }
    // T_EE E_u E_v + T_EV (E_u V_v + V_u E_v) = E_u a_v + c_u E_v with a = T_EE E + T_EV V,
    // c = T_EV V
    T av[kPrim], cu[kPrim];
#pragma unroll
    for (int u = 0; u < kPrim; ++u) {
      G[u] = fma(cE, Eu[u], fma(cV, Vu[u], G[u]));
      av[u] = fma(TEE, Eu[u], TEV * Vu[u]);
      cu[u] = TEV * Vu[u];
    }
#pragma unroll
    for (int u = 0; u < kPrim; ++u) {
#pragma unroll
      for (int v = u; v < kPrim; ++v) {
        // E_u vanishes in the two amplitude-variance coordinates (u = 3, 4)
        T q = Q[qidx(u, v)];
        if (v != 3 && v != 4) q = fma(cu[u], Eu[v], q);
        if (u != 3 && u != 4) q = fma(Eu[u], av[v], q);
        Q[qidx(u, v)] = q;
      }
    }
    // second derivatives of E_s and V_s
    Q[qidx(0, 0)] += cV * (T)-2 * d * d;
    Q[qidx(0, 1)] += fma(cE, -f0, cV * ((T)-2 * L0 * e0 * f0 * f0 + (T)2 * oma2 * d * f0));
    Q[qidx(0, 2)] += fma(cE, f1, cV * ((T)2 * L1 * e1 * f1 * f1 - (T)2 * oma2 * d * f1));
    Q[qidx(0, 3)] += cV * (-L0 * L0 * f0 * f0);
    Q[qidx(0, 4)] += cV * (L1 * L1 * f1 * f1);
    Q[qidx(1, 1)] += cV * ((T)2 * w0 * e0 * f0 * f0 + (T)2 * w01 * f0 * f0);
    Q[qidx(1, 2)] += cV * ((T)-2 * w01 * f0 * f1);
    Q[qidx(1, 3)] += cV * ((T)2 * w0 * L0 * f0 * f0);
    Q[qidx(2, 2)] += cV * ((T)2 * w1 * e1 * f1 * f1 + (T)2 * w01 * f1 * f1);
    Q[qidx(2, 4)] += cV * ((T)2 * w1 * L1 * f1 * f1);
    // the (amplitude, z) pairs are linear in g0, g1 and dz with weights fixed per pixel:
    //   Q[0][z] += c_E (-dz) + c_V (-2 L0^2 e0 f0 g0 + 2 L1^2 e1 f1 g1 + 2 (1 - 2a) d dz)
    //   Q[1][z] += c_E w0 g0 + c_V (4 w0 L0 e0 f0 g0 + 2 w01 (f0 dz + d g0))
    //   Q[2][z] += c_E w1 g1 + c_V (4 w1 L1 e1 f1 g1 - 2 w01 (f1 dz + d g1))
    //   Q[3][z] += c_V 2 w0 L0^2 f0 g0,  Q[4][z] += c_V 2 w1 L1^2 f1 g1
    const T a0 = -cV2 * L0 * L0 * e0 * f0, b0 = cV2 * L1 * L1 * e1 * f1, c0 = fma(cV2 * oma2, d, -cE);
    const T a1 = fma(cE, w0, cV2 * fma((T)2 * w0 * L0 * e0, f0, w01 * d)), c1 = cV2 * w01 * f0;
    const T b2 = fma(cE, w1, cV2 * fma((T)2 * w1 * L1 * e1, f1, -w01 * d)), c2 = -cV2 * w01 * f1;
    const T a3 = cV2 * w0 * L0 * L0 * f0, b4 = cV2 * w1 * L1 * L1 * f1;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const T g0j = o.g0[j], dzj = dz[j];
      T q0 = fma(a0, g0j, fma(c0, dzj, Q[qidx(0, 5 + j)]));
      T q1 = fma(a1, g0j, fma(c1, dzj, Q[qidx(1, 5 + j)]));
      T q2 = fma(c2, dzj, Q[qidx(2, 5 + j)]);
      if (j < 2) {
        q0 = fma(b0, g1z[j], q0);
        q2 = fma(b2, g1z[j], q2);
        Q[qidx(4, 5 + j)] = fma(b4, g1z[j], Q[qidx(4, 5 + j)]);
      }
      Q[qidx(0, 5 + j)] = q0;
      Q[qidx(1, 5 + j)] = q1;
      Q[qidx(2, 5 + j)] = q2;
      Q[qidx(3, 5 + j)] = fma(a3, g0j, Q[qidx(3, 5 + j)]);
    }
    col += step_cols;
    row += step_rows;
    if (col >= P.w) {
      col -= P.w;
      row += 1;
    }
  }
  // the slot row's 79 wavefront sums, formed together in two groups (the first 64 of the 77
  // first- and second-order sums, exchanged in the pixel precision at the first step; then
  // the two objective sums with the last 13); the lane holding a sum stores it
  double* out = a.hslots + (int64_t)t * kHSlots;
  constexpr int kGQ = kPrim + kHQ, kA = 64, kB = 2 + kGQ - kA;
  {
    T v[kA];
#pragma unroll
    for (int i = 0; i < kA; ++i) v[i] = i < kPrim ? G[i] : Q[i - kPrim];
    const double sv = wave_sums<kA, 32, T>(v, lane);
    const int sl = wave_sums_slot<kA>(lane);
    if (sl >= 0) out[2 + sl] = sv;
  }
  {
    double v[kB];
    v[0] = tsum;
    v[1] = town;
#pragma unroll
    for (int i = 2; i < kB; ++i) v[i] = (double)Q[kA + i - 2 - kPrim];
    const double sv = wave_sums<kB>(v, lane);
    const int sl = wave_sums_slot<kB>(lane);
    if (sl >= 0) out[sl < 2 ? sl : kA + sl] = sv;
  }
}

// Sigma_s(angle, log r, logit axis) and its first and second derivatives in those three
// coordinates (Section 2.1.2): out d1[t][e], d2[t][t'][e] with e = (xx, xy, yy).
__device__ void sigma_derivs(double ang, double lr, double eta, double d1[3][3], double d2[3][3][3]) {
  const double c = cos(ang), s = sin(ang), r2 = exp(2.0 * lr), rho = sigmoid(eta);
  const double rp = rho * (1.0 - rho), rpp = rp * (1.0 - 2.0 * rho);
  const double sig[3] = {r2 * (c * c + rho * rho * s * s), r2 * (rho * rho - 1.0) * c * s,
                         r2 * (s * s + rho * rho * c * c)};
  const double dt[3] = {2.0 * r2 * c * s * (rho * rho - 1.0), r2 * (rho * rho - 1.0) * (c * c - s * s),
                        -2.0 * r2 * c * s * (rho * rho - 1.0)};
  const double dtt[3] = {2.0 * r2 * (rho * rho - 1.0) * (c * c - s * s), -4.0 * r2 * (rho * rho - 1.0) * c * s,
                         -2.0 * r2 * (rho * rho - 1.0) * (c * c - s * s)};
  const double dr[3] = {2.0 * rho * r2 * s * s, 2.0 * rho * r2 * c * s, 2.0 * rho * r2 * c * c};
  const double drr[3] = {2.0 * r2 * s * s, 2.0 * r2 * c * s, 2.0 * r2 * c * c};
  const double dtr[3] = {4.0 * rho * r2 * c * s, 2.0 * rho * r2 * (c * c - s * s), -4.0 * rho * r2 * c * s};
  for (int e = 0; e < 3; ++e) {
    d1[0][e] = dt[e];
    d1[1][e] = 2.0 * sig[e];
    d1[2][e] = dr[e] * rp;
    d2[0][0][e] = dtt[e];
    d2[1][1][e] = 4.0 * sig[e];
    d2[2][2][e] = drr[e] * rp * rp + dr[e] * rpp;
    d2[0][1][e] = d2[1][0][e] = 2.0 * dt[e];
    d2[1][2][e] = d2[2][1][e] = 2.0 * dr[e] * rp;
    d2[0][2][e] = d2[2][0][e] = dtr[e] * rp;
  }
}

// S = A M A^T for a symmetric M given as (xx, xy, yy)
__device__ __forceinline__ void conj_A(const double A[2][2], const double* m, double* out) {
  const double t00 = A[0][0] * m[0] + A[0][1] * m[1], t01 = A[0][0] * m[1] + A[0][1] * m[2];
  const double t10 = A[1][0] * m[0] + A[1][1] * m[1], t11 = A[1][0] * m[1] + A[1][1] * m[2];
  out[0] = t00 * A[0][0] + t01 * A[0][1];
  out[1] = t00 * A[1][0] + t01 * A[1][1];
  out[2] = t10 * A[1][0] + t11 * A[1][1];
}

struct HessFinArgs {
  const int32_t* job_src;
  int32_t n_jobs;
  const uint8_t* active;
  const double* theta;
  const double* hslots;
  const int32_t* patch_ptr;
  const DPatch* patches;
  const double* pix_const;
  const cel_image* images;
  const DPrior* prior;
  int32_t with_kl;             // 1: the Hessian includes the KL part (value and gradient always do)
  double* local;               // [S]
  double* grad;                // [S][32]
  double* hess;                // [S][27][27]
  int32_t* err;                // device condition word (non-finite Hessian entries)
  double* part;                // [S][kHParts][kPartN] per-part sums: Hessian, gradient, local
};

// The pixel part of a source's Hessian is summed over its patches by kHParts wavefronts,
// each taking a contiguous quarter of the patches (a single wavefront per source leaves
// most SIMDs idle and waits on every latency alone); k_hess_combine adds the parts in a
// fixed order and the KL terms.
constexpr int kHParts = kHessParts;
constexpr int kPartN = kHessPartN;   // Hessian, gradient, local, pad
static_assert(kPartN >= kN * kN + kN + 1, "part record too small");

// Sparsity of J = dr/dtheta (r: the 11 primitive coordinates, theta: the 27 parameters):
// column k has jcount(k) nonzero rows jrow(k, e) -- the centre rows for the position, the
// flux rows m_i / v_i for the flux and colour parameters, the three S rows for the angle,
// radius and axis, and one row each for the type and profile logits.
__device__ __forceinline__ int jcount(int k) { return k < 2 ? 2 : (k == 23 || k == 24 || k == 26) ? 3 : 1; }
__device__ __forceinline__ int jrow(int k, int e) {
  if (k < 2) return 5 + e;
  if (k == 2) return 0;
  if (k < 5) return 1 + 2 * (k - 3);
  if (k < 7) return 2 + 2 * (k - 5);
  if (k < 15) return 1 + 2 * ((k - 7) / 4);
  if (k < 23) return 2 + 2 * ((k - 15) / 4);
  if (k == 25) return 10;
  return 7 + e;
}

__global__ __launch_bounds__(64) void k_hess_finalize(HessFinArgs a) {
  const int s = a.job_src ? a.job_src[blockIdx.x] : (int)blockIdx.x;
  if (a.active && !a.active[s]) return;
  const int lane = threadIdx.x;
  const int w = blockIdx.y;
  // slot sums and flux moments of up to kPB patches, gathered together (one memory and one
  // exp latency per batch instead of per patch)
  constexpr int kPB = 16, kHU = 2 + kPrim + kHQ;
  __shared__ double smb[kPB][kHU], Lfb[kPB][2], evb[kPB][2];
  __shared__ double Qr[kPrim][kPrim], Gr[kPrim];
  // column k of dr/dtheta: rows jr[k][e] with values jv[k][e] (zero past jcount(k)); dg the
  // diagonal and sblk the S-block second-derivative terms
  __shared__ double jv[kN][3], dg[kN], sblk[3][3];
  __shared__ int jr[kN][3];
  __shared__ double gs[kThetaN];
  __shared__ double th[kN], sd1[3][3], sd2[3][3][3];
  __shared__ double rv[2], cvv[2][4];
  if (lane < kN) th[lane] = a.theta[(int64_t)s * kThetaN + lane];
  if (lane < kThetaN) gs[lane] = 0.0;
  __syncthreads();
  if (lane == 0) sigma_derivs(th[23], th[24], th[26], sd1, sd2);
  if (lane < kN) {
#pragma unroll
    for (int e = 0; e < 3; ++e) jr[lane][e] = e < jcount(lane) ? jrow(lane, e) : jrow(lane, 0);
  }
  // flux and colour variances, one per lane
  if (lane >= 1 && lane < 11) {
    const int l = lane - 1;
    const double e = exp(l < 2 ? th[5 + l] : th[15 + (l - 2)]);
    if (l < 2) rv[l] = e;
    else cvv[(l - 2) / 4][(l - 2) % 4] = e;
  }
  __syncthreads();
  // this lane's Hessian entries idx = lane + 64 m accumulate in registers over the patches
  constexpr int kHPer = (kN * kN + 63) / 64;
  double hacc[kHPer];
#pragma unroll
  for (int m = 0; m < kHPer; ++m) hacc[m] = 0.0;
  double local = 0.0;
  const double aa = sigmoid(th[2]), pi = sigmoid(th[25]);
  // this part's patches: a contiguous share of the source's
  const int q0 = a.patch_ptr[s], nq = a.patch_ptr[s + 1] - q0, per = (nq + kHParts - 1) / kHParts;
  const int p0 = q0 + min(nq, w * per), p1 = q0 + min(nq, (w + 1) * per);
  for (int pb = p0; pb < p1; pb += kPB) {
    const int nb = min(kPB, p1 - pb);
    for (int e = lane; e < nb * kHU; e += 64) {
      const int q = e / kHU, l = e % kHU;
      const DPatch P = a.patches[pb + q];
      double acc = 0;
      for (int t = P.task_begin; t < P.task_end; ++t) acc += a.hslots[(int64_t)t * kHSlots + l];
      smb[q][l] = acc;
    }
    // flux moments of each patch's band: L_i = iota exp(m_i + v_i / 2) and e_i = exp(v_i),
    // lane 4 q + 2 w + i
    if (lane < 4 * nb) {
      const int q = lane >> 2, i = lane & 1, w = (lane >> 1) & 1;
      const cel_image& imq = a.images[a.patches[pb + q].img];
      double m = th[3 + i], var = rv[i];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double W = c_W[imq.band][c];
        m += W * th[7 + 4 * i + c];
        var += W * W * cvv[i][c];
      }
      const double ex = exp(w == 0 ? m + 0.5 * var : var);
      if (w == 0) Lfb[q][i] = imq.iota * ex;
      else evb[q][i] = ex;
    }
    __syncthreads();
    for (int q = 0; q < nb; ++q) {
      const int p = pb + q;
      const DPatch P = a.patches[p];
      const cel_image& im = a.images[P.img];
      const double* sm = smb[q];
      const double* Lf = Lfb[q];
      const double* ev = evb[q];
      local += sm[0] + a.pix_const[2 * p];
      // stage 1: y = (a, L0, L1, e0, e1, z) -> r = (a, m0, v0, m1, v1, z).  Each r is reached
      // from at most two y: a <- a; m_i <- L_i (dL/dm = L); v_i <- L_i (L/2) and e_i (e^v);
      // z <- z.  Qr = Jy^T Qy Jy + sum_u g_u d2y_u/dr2, Gr = Jy^T g.  Written without
      // branches: the second source of an r that has one is given weight 0.
      auto ysrc = [&](int r, int* u, double* j) {
        const bool flux = r >= 1 && r <= 4;
        const int i = (r - 1) >> 1;
        const bool var = flux && ((r & 1) == 0);
        const double L = i ? Lf[1] : Lf[0], e = i ? ev[1] : ev[0];
        u[0] = flux ? 1 + i : r;
        j[0] = flux ? (var ? 0.5 * L : L) : 1.0;
        u[1] = var ? 3 + i : u[0];
        j[1] = var ? e : 0.0;
      };
      for (int idx = lane; idx < kPrim * kPrim; idx += 64) {
        const int r = idx / kPrim, r2 = idx % kPrim;
        int ua[2], ub[2];
        double ja[2], jb[2];
        ysrc(r, ua, ja);
        ysrc(r2, ub, jb);
        double v = 0;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const int u = ua[x], w = ub[y];
            v += ja[x] * sm[2 + kPrim + (u <= w ? qidx(u, w) : qidx(w, u))] * jb[y];
          }
        // second derivatives of y in r: L_i: mm = L, mv = L/2, vv = L/4; e_i: vv = e^v
        if (r >= 1 && r <= 4 && r2 >= 1 && r2 <= 4 && ((r - 1) >> 1) == ((r2 - 1) >> 1)) {
          const int i = (r - 1) >> 1;
          const double gL = sm[3 + i], ge = sm[5 + i];
          const double L = i ? Lf[1] : Lf[0], e = i ? ev[1] : ev[0];
          const int nv = ((r & 1) == 0) + ((r2 & 1) == 0);   // how many of r, r2 are v_i
          v += gL * L * (nv == 0 ? 1.0 : nv == 1 ? 0.5 : 0.25) + (nv == 2 ? ge * e : 0.0);
        }
        Qr[r][r2] = v;
      }
      if (lane < kPrim) {
        int ua[2];
        double ja[2];
        ysrc(lane, ua, ja);
        Gr[lane] = ja[0] * sm[2 + ua[0]] + ja[1] * sm[2 + ua[1]];
      }
      __syncthreads();   // Gr is read below
      // stage 2: the nonzero values of column k of J = dr/dtheta (zero-padded to 3), all
      // candidates formed and one selected
      if (lane < kN) {
        const int k = lane;
        const double A00 = im.A[0][0], A01 = im.A[0][1], A10 = im.A[1][0], A11 = im.A[1][1];
        const int c = (k - 7) & 3, ti = (k - 15) >> 2;
        const double W = c_W[im.band][c];
        const int t = k == 23 ? 0 : k == 24 ? 1 : 2;
        double sv[3];
        conj_A(im.A, sd1[t], sv);
        const bool sk = k == 23 || k == 24 || k == 26;
        double v0 = 0.0;
        v0 = k == 0 ? A00 : k == 1 ? A01 : v0;
        v0 = k == 2 ? aa * (1.0 - aa) : v0;
        v0 = (k == 3 || k == 4) ? 1.0 : v0;
        v0 = (k == 5 || k == 6) ? rv[k == 6] : v0;
        v0 = (k >= 7 && k < 15) ? W : v0;
        v0 = (k >= 15 && k < 23) ? W * W * cvv[ti & 1][c] : v0;
        v0 = k == 25 ? pi * (1.0 - pi) : v0;
        v0 = sk ? sv[0] : v0;
        jv[k][0] = v0;
        jv[k][1] = k == 0 ? A10 : k == 1 ? A11 : sk ? sv[1] : 0.0;
        jv[k][2] = sk ? sv[2] : 0.0;
        // the diagonal second-derivative terms sum_r Gr[r] d2r/dtheta_k^2 (outside the S block)
        double dgk = 0.0;
        dgk = k == 2 ? Gr[0] * aa * (1.0 - aa) * (1.0 - 2.0 * aa) : dgk;
        dgk = (k == 5 || k == 6) ? Gr[2 + 2 * (k - 5)] * rv[k == 6] : dgk;
        dgk = (k >= 15 && k < 23) ? Gr[2 + 2 * (ti & 1)] * W * W * cvv[ti & 1][c] : dgk;
        dgk = k == 25 ? Gr[10] * pi * (1.0 - pi) * (1.0 - 2.0 * pi) : dgk;
        dg[k] = dgk;
      }
      // S block (angle, radius, axis): sum_r Gr[r] d2S_r/dt dt'
      if (lane >= 32 && lane < 41) {
        const int ti = (lane - 32) / 3, tk = (lane - 32) % 3;
        double sv[3];
        conj_A(im.A, sd2[ti][tk], sv);
        sblk[ti][tk] = Gr[7] * sv[0] + Gr[8] * sv[1] + Gr[9] * sv[2];
      }
      __syncthreads();
      // H += J^T Qr J + the second-derivative terms, 3 x 3 terms per entry (zero-padded
      // columns; the rows of column k are jr[k][e])
#pragma unroll
      for (int m = 0; m < kHPer; ++m) {
        const int idx = lane + 64 * m;
        if (idx >= kN * kN) break;
        const int i = idx / kN, k = idx % kN;
        double v = 0;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          const int r = jr[i][x];
          double tt = 0;
#pragma unroll
          for (int y = 0; y < 3; ++y) tt += Qr[r][jr[k][y]] * jv[k][y];
          v += jv[i][x] * tt;
        }
        if (i == k) v += dg[i];
        const int si = i == 23 ? 0 : i == 24 ? 1 : i == 26 ? 2 : -1;
        const int sk = k == 23 ? 0 : k == 24 ? 1 : k == 26 ? 2 : -1;
        if (si >= 0 && sk >= 0) v += sblk[si][sk];
        hacc[m] += v;
      }
      if (lane < kN) gs[lane] += jv[lane][0] * Gr[jr[lane][0]] + jv[lane][1] * Gr[jr[lane][1]] + jv[lane][2] * Gr[jr[lane][2]];
      __syncthreads();
    }
  }
  // this part's sums
  double* out = a.part + ((int64_t)s * kHParts + w) * kPartN;
#pragma unroll
  for (int m = 0; m < kHPer; ++m) {
    const int idx = lane + 64 * m;
    if (idx < kN * kN) out[idx] = hacc[m];
  }
  __syncthreads();   // gs is complete
  if (lane < kN) out[kN * kN + lane] = gs[lane];
  if (lane == 0) out[kN * kN + kN] = local;   // (every lane holds the same sum)
}

// one wavefront per source: the parts' sums in a fixed order, then the KL value, gradient
// and (with with_kl) Hessian, and the outputs
__global__ __launch_bounds__(64) void k_hess_combine(HessFinArgs a) {
  const int s = a.job_src ? a.job_src[blockIdx.x] : (int)blockIdx.x;
  if (a.active && !a.active[s]) return;
  const int lane = threadIdx.x;
  __shared__ double Hs[kN][kLd], gs[kThetaN], th[kN];
  if (lane < kN) th[lane] = a.theta[(int64_t)s * kThetaN + lane];
  const double* part = a.part + (int64_t)s * kHParts * kPartN;
  for (int idx = lane; idx < kN * kN; idx += 64) {
    double h = 0.0;
#pragma unroll
    for (int w = 0; w < kHParts; ++w) h += part[w * kPartN + idx];
    Hs[idx / kN][idx % kN] = h;
  }
  if (lane < kThetaN) {
    double g = 0.0;
    if (lane < kN)
#pragma unroll
      for (int w = 0; w < kHParts; ++w) g += part[w * kPartN + kN * kN + lane];
    gs[lane] = g;
  }
  double local = 0.0;
#pragma unroll
  for (int w = 0; w < kHParts; ++w) local += part[w * kPartN + kN * kN + kN];
  __syncthreads();
  // KL: value, gradient and (optionally) Hessian
  __shared__ double klv;
  {
    double gk[kThetaN];
#pragma unroll
    for (int k = 0; k < kThetaN; ++k) gk[k] = 0.0;
    const double kv = kl_source_wave(*a.prior, th, gk, 1.0, lane);   // every lane: gk = -grad KL
    if (lane == 0) {
      klv = kv;
#pragma unroll
      for (int k = 0; k < kN; ++k) gs[k] += gk[k];
    }
  }
  if (a.with_kl) {
    __shared__ double klw[16][kKlw], kls[2][kKlw];
    kl_hessian_wave<kLd>(*a.prior, th, Hs, -1.0, lane, klw, kls);
  }
  __syncthreads();
  if (lane == 0 && a.local) a.local[s] = local - klv;
  if (a.grad && lane < kThetaN) a.grad[(int64_t)s * kThetaN + lane] = lane < kN ? gs[lane] : 0.0;
  bool fin = true;
  for (int idx = lane; idx < kN * kN; idx += 64) {
    const double h = Hs[idx / kN][idx % kN];
    fin = fin && isfinite(h);
    a.hess[(int64_t)s * kN * kN + idx] = h;
  }
  if (a.err && !fin) atomicOr(a.err, CEL_DEVERR_NONFINITE_HESSIAN);
}

struct TrArgs {
  const int32_t* job_src;     // sources of this launch
  int32_t n_jobs;
  const uint8_t* active;
  const double* v_grad;       // gradient at the iterate [S][32]
  const double* v_local;      // L_s at the iterate [S]
  const double* hess;         // Hessian of L_s [S][27][27]
  const double* theta;
  const double* radius;
  const double* npix;         // active pixels per source
  double gtol, ftol, radius_min;
  double* theta_trial;        // out [S][32]
  uint8_t* trial_active;      // out: 1 = trial point to evaluate
  double* pred;               // out: predicted gain
  double* pnorm;              // out: |p|
  int32_t* status;            // out: CONVERGED / NONFINITE for sources not tried
  int32_t* err;               // device condition word
};

// Hessian of L_s from central differences of the pixel gradient (variants 1..54 hold the
// gradients at theta_s +/- h e_k), symmetrised, minus the analytic KL Hessian (the tight
// colour-prior mixture makes the KL's higher derivatives too large for differencing).
struct FdHessArgs {
  const int32_t* job_src;
  int32_t n_jobs, S;
  const uint8_t* active;
  const double* v_grad;       // [variants][S][32]
  double fd_step;
  const double* theta;
  const DPrior* prior;
  double* hess;               // out [S][27][27]
};

__global__ __launch_bounds__(64) void k_fd_hessian(FdHessArgs a) {
  const int s = a.job_src ? a.job_src[blockIdx.x] : (int)blockIdx.x;
  if (a.active && !a.active[s]) return;
  const int lane = threadIdx.x;
  __shared__ double H[kN][kLd];
  __shared__ double th[kN];
  const int64_t vs = (int64_t)a.S * kThetaN;
  const double h2 = 2.0 * a.fd_step;
  for (int idx = lane; idx < kN * kN; idx += 64) {
    const int i = idx / kN, k = idx % kN;
    const double hik = (a.v_grad[(int64_t)(1 + k) * vs + (int64_t)s * kThetaN + i] -
                        a.v_grad[(int64_t)(1 + kN + k) * vs + (int64_t)s * kThetaN + i]) / h2;
    const double hki = (a.v_grad[(int64_t)(1 + i) * vs + (int64_t)s * kThetaN + k] -
                        a.v_grad[(int64_t)(1 + kN + i) * vs + (int64_t)s * kThetaN + k]) / h2;
    H[i][k] = 0.5 * (hik + hki);
  }
  if (lane < kN) th[lane] = a.theta[(int64_t)s * kThetaN + lane];
  __syncthreads();
  __shared__ double klw[16][kKlw], kls[2][kKlw];
  kl_hessian_wave<kLd>(*a.prior, th, H, -1.0, lane, klw, kls);
  for (int idx = lane; idx < kN * kN; idx += 64) a.hess[(int64_t)s * kN * kN + idx] = H[idx / kN][idx % kN];
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Eigen-decomposition for the trust-region subproblem: one-sided (Hestenes) Jacobi on
// W = B + c I, c = 1.001 |B|_F (positive definite, so its singular vectors are B's
// eigenvectors and its singular values the shifted eigenvalues).  Lane k holds column k of
// W in registers; in round r of a sweep the lanes pair up by the round-robin (circle)
// schedule -- columns (r + m, r - m) mod 27 for m = 1..13, column r with the zero column 27
// -- exchange columns with one shuffle per entry, and orthogonalise each pair by the
// rotation that diagonalises its 2x2 Gram block.  Sweeps stop when a whole sweep finds
// every pair orthogonal to 1e-15; then lambda_k = |w_k| - c and v_k = w_k / |w_k|.
__global__ __launch_bounds__(64) void k_trsolve(TrArgs a) {
  const int s = a.job_src ? a.job_src[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x, lane = tid;
  if (a.active && !a.active[s]) {
    if (tid == 0) a.trial_active[s] = 0;
    return;
  }
  __shared__ double B[kN][kLd];
  __shared__ double V[kN][kLd];
  __shared__ double g[kN], lam[kN], y[kN], gt[kN];
  __shared__ int outcome;   // 0 continue, 1 non-finite, 2 converged
  const double L = a.v_local[s];
  const double radius = a.radius[s];
  // B = -H (the Hessian of L_s, pixel and KL parts), symmetrised
  for (int idx = tid; idx < kN * kN; idx += 64) {
    const int i = idx / kN, k = idx % kN;
    B[i][k] = -0.5 * (a.hess[(int64_t)s * kN * kN + i * kN + k] + a.hess[(int64_t)s * kN * kN + k * kN + i]);
  }
  if (tid < kN) g[tid] = a.v_grad[(int64_t)s * kThetaN + tid];
  __syncthreads();
  // finiteness and the gradient test (wave reductions: every lane holds the same result)
  double bad = 0.0, gm = 0.0, fro = 0.0;
  for (int idx = lane; idx < kN * kN; idx += 64) {
    const double b = B[idx / kN][idx % kN];
    if (!isfinite(b)) bad = 1.0;
    fro += b * b;
  }
  if (lane < kN) {
    if (!isfinite(g[lane])) bad = 1.0;
    gm = fabs(g[lane]);
  }
  bad = wave_max(bad);
  const double gmax = wave_max(gm);
  fro = wave_sum<double>(fro);
  if (bad != 0.0 || !isfinite(L) || !isfinite(radius)) {
    if (lane == 0) {
      a.status[s] = CEL_ST_NONFINITE;
      a.trial_active[s] = 0;
      if (a.err) atomicOr(a.err, CEL_DEVERR_NONFINITE_STEP);
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
  const double cs = sqrt(fro) * 1.001 + 1e-300;
  // Lane 32 h + c holds rows 14 h .. 14 h + 13 of column c (c < 27; column 27 is the idle
  // partner of the odd-size round-robin), so a round exchanges and rotates 14 entries per
  // lane; sums over a column add the two halves (lanes c and c + 32).
  constexpr int kH = (kN + 1) / 2;
  const int half = lane >> 5, col = lane & 31;
  auto hsum = [&](double v) { return v + __shfl_xor(v, 32, 64); };
  double w[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    const int row = half * kH + i;
    w[i] = (col < kN && row < kN) ? B[row][col] + (row == col ? cs : 0.0) : 0.0;
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    double rotated = 0.0;
    // squared column norm, exact at the start of a sweep and carried through its rotations
    // (|c w + cp pw|^2 = c^2 al + cp^2 be + 2 c cp ga)
    double al;
    {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int i = 0; i < kH; i += 2) {
        a0 = fma(w[i], w[i], a0);
        a1 = fma(w[i + 1], w[i + 1], a1);
      }
      al = hsum(a0 + a1);
    }
    for (int r = 0; r < kN; ++r) {
      const int pc = col > kN ? col : col == kN ? r : col == r ? kN : ((2 * r - col) % kN + kN) % kN;
      const int pt = half * 32 + pc;
      double pw[kH];
      const double be = __shfl(al, pt, 64);
#pragma unroll
      for (int i = 0; i < kH; ++i) pw[i] = __shfl(w[i], pt, 64);
      double g0 = 0.0, g1 = 0.0;   // two chains for the dot product
#pragma unroll
      for (int i = 0; i < kH; i += 2) {
        g0 = fma(w[i], pw[i], g0);
        g1 = fma(w[i + 1], pw[i + 1], g1);
      }
      const double ga = hsum(g0 + g1);
      const bool lowside = col < pc;
      const double alo = lowside ? al : be, ahi = lowside ? be : al;
      double c = 1.0, sn = 0.0;
      // the pair is rotated unless orthogonal to 1e-15 of its norms' product
      // (|ga| > 1e-15 sqrt(alo ahi), compared squared)
      if (ga * ga > 1e-30 * (alo * ahi)) {
        // t = tan of the rotation angle, the root of smaller magnitude of t^2 + 2 zeta t - 1 = 0
        // with zeta = (ahi - alo) / (2 ga), written without zeta: with d = ahi - alo,
        // t = sign(d) 2 ga / (|d| + sqrt(d^2 + 4 ga^2)) (d = 0: t = sign(ga), both roots of
        // size 1 annihilate the pair); c = 1 / sqrt(1 + t^2), |t| <= 1
        const double d = ahi - alo;
        const double r = sqrt(fma(d, d, 4.0 * ga * ga));
        const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + r);
        c = rsqrt(fma(t, t, 1.0));
        sn = c * t;
        rotated = 1.0;
      }
      const double cp = lowside ? -sn : sn;
#pragma unroll
      for (int i = 0; i < kH; ++i) w[i] = fma(c, w[i], cp * pw[i]);
      al = c * c * al + cp * cp * be + 2.0 * c * cp * ga;
    }
    if (wave_max(rotated) == 0.0) break;
  }
  {
    double nn = 0.0;
#pragma unroll
    for (int i = 0; i < kH; ++i) nn = fma(w[i], w[i], nn);
    const double sig = sqrt(hsum(nn)), inv = 1.0 / sig;
    double acc = 0.0;   // gt = V^T g
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      const int row = half * kH + i;
      if (col < kN && row < kN) {
        const double v = w[i] * inv;
        V[row][col] = v;
        acc = fma(v, g[row], acc);
      }
    }
    acc = hsum(acc);
    if (col < kN && half == 0) {
      lam[col] = sig - cs;
      gt[col] = acc;
    }
  }
  __syncthreads();
  bool go = false;
  {
  // the trust-region subproblem in the eigenbasis; scalar logic runs identically on every
  // lane, sums over the 27 eigenvalues are wave reductions
  const bool own = lane < kN;
  const double lam_l = own ? lam[lane] : 0.0, gt_l = own ? gt[lane] : 0.0;
  const double gnorm = sqrt(wave_sum<double>(own ? g[lane] * g[lane] : 0.0));
  double lmin = lam[0];
  int imin = 0;
  for (int i = 1; i < kN; ++i)
    if (lam[i] < lmin) {
      lmin = lam[i];
      imin = i;
    }
  const bool low_l = own && fabs(lam_l - lmin) <= 1e-12 * fmax(1.0, fabs(lmin));
  // shifted eigenvalues d_i = lam_i + lo >= 0 (exact zero at the lowest): the multiplier is
  // lo + mu, and |p|^2 = sum gt_i^2 / (d_i + mu)^2 keeps its precision near the pole
  const double lo = fmax(0.0, -lmin);
  const double dl = own ? lam_l + lo : 0.0;
  auto norm_mu = [&](double m) {
    const double v = own ? gt_l / (dl + m) : 0.0;
    return sqrt(wave_sum<double>(v * v));
  };
  double mu = -1.0;   // chosen shifted multiplier (< 0: not yet found)
  bool hard = false;
  if (lmin > 0 && norm_mu(0.0) <= radius) mu = 0.0;
  double tau_hard = 0.0;
  if (mu < 0) {
    const double notorth = wave_max((low_l && fabs(gt_l) > 1e-12 * fmax(gnorm, 1e-300)) ? 1.0 : 0.0);
    if (notorth == 0.0) {
      const double v = (own && !low_l) ? gt_l / dl : 0.0;
      const double nr = wave_sum<double>(v * v);
      if (sqrt(nr) <= radius) {
        hard = true;
        mu = 0.0;
        tau_hard = sqrt(fmax(radius * radius - nr, 0.0));
      }
    }
  }
  if (mu < 0) {
    // boundary multiplier: |p| = radius for mu in (0, inf).  Safeguarded Newton on
    // 1/radius - 1/|p|, convex and decreasing in mu (Nocedal & Wright, Algorithm 4.3, in
    // the eigenbasis: |q|^2 = sum gt_i^2 / (d_i + mu)^3), inside a bracket [aa, bb] with
    // |p(aa)| > radius >= |p(bb)|, bisecting when a step leaves it; 4-13 steps to
    // |p| = radius (1 + O(eps)).
    double hi = gnorm / radius + 1.0;
    while (norm_mu(hi) > radius) hi *= 2.0;
    double aa = 0.0, bb = hi;
    const double glow = wave_max(low_l ? fabs(gt_l) : 0.0);
    double mc = lmin > 0 ? 0.0 : 0.5 * glow / radius;   // left of the root
    if (!(mc >= aa && mc < bb) || (lmin <= 0 && !(mc > 0.0))) mc = 0.5 * (aa + bb);
    for (int it = 0; it < 200 && mu < 0; ++it) {
      const double v = own ? 1.0 / (dl + mc) : 0.0;
      const double pv = gt_l * v;
      const double s1 = wave_sum<double>(pv * pv), s2 = wave_sum<double>(pv * pv * v);
      const double np = sqrt(s1);
      if (np > radius) aa = mc;
      else bb = mc;
      double nx = mc + (s1 / s2) * (np - radius) / radius;
      if (!(nx > aa && nx < bb)) nx = 0.5 * (aa + bb);
      if (fabs(np - radius) <= 4.0 * DBL_EPSILON * radius || nx == mc) mu = mc;   // converged
      else if (bb - aa <= 4.0 * DBL_EPSILON * bb) mu = bb;                        // bracket closed
      mc = nx;
    }
    if (mu < 0) mu = bb;
  }
  // step in the eigenbasis (hard case: completed along the lowest eigenvector, oriented so
  // that its largest-magnitude entry is positive), predicted gain and norm
  double yl = 0.0;
  if (own) yl = (hard && low_l) ? 0.0 : gt_l / (dl + mu);
  if (hard && lane == imin) {
    int am = 0;
    for (int i = 1; i < kN; ++i)
      if (fabs(V[i][imin]) > fabs(V[am][imin])) am = i;
    yl = V[am][imin] < 0 ? -tau_hard : tau_hard;
  }
  const double gp = wave_sum<double>(gt_l * yl), pBp = wave_sum<double>(lam_l * yl * yl), nn = wave_sum<double>(yl * yl);
  if (own) y[lane] = yl;
  const double pr = gp - 0.5 * pBp;
  go = pr > a.ftol * fmax(1.0, fabs(L));
  if (lane == 0) {
    a.pred[s] = pr;
    a.pnorm[s] = sqrt(nn);
    if (!go) a.status[s] = CEL_ST_CONVERGED;
    a.trial_active[s] = go ? 1 : 0;
    outcome = go ? 0 : 2;
  }
  }
  __syncthreads();
  if (outcome) return;
  if (tid < kThetaN) {
    double v = a.theta[(int64_t)s * kThetaN + tid];
    if (tid < kN) {
      double step = 0;
      for (int i = 0; i < kN; ++i) step += V[tid][i] * y[i];
      v += step;
    }
    a.theta_trial[(int64_t)s * kThetaN + tid] = v;
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

template <typename T>
static hipError_t launch_hess_t(cel_plan* p, const int32_t* order, int n_items, const uint8_t* active,
                                hipStream_t sm) {
  if (n_items <= 0) return hipSuccess;
  HessArgs ha;
  std::memset(&ha, 0, sizeof(ha));
  ha.tasks = p->d_tasks;
  ha.order = order;
  ha.patches = p->d_patches;
  ha.nbr_idx = p->d_nbr;
  ha.tables = sizeof(T) == 8 ? (const void*)p->tables_d : (const void*)p->tables_f;
  ha.xs = sizeof(T) == 8 ? (const void*)p->d_xs64 : (const void*)p->d_xs;
  ha.maps = sizeof(T) == 8 ? (const void*)p->d_maps64 : (const void*)p->d_maps;
  ha.hslots = p->d_hslots;
  ha.active = active;
  ha.img_npsf = p->d_npsf;
  if (p->nexp == 6 && p->ndev == 8)
    hipLaunchKernelGGL((k_hess<T, 6, 8>), dim3(n_items), dim3(64), 0, sm, ha);
  else
    hipLaunchKernelGGL((k_hess<T, 8, 8>), dim3(n_items), dim3(64), 0, sm, ha);
  return hipGetLastError();
}

// Analytic per-source Hessians (pixel part, plus the KL part when with_kl) of the sources
// flagged in `active` among `srcs` (device list, n_src entries; null = 0..S-1), with their
// gradients and local objectives.  The base tables and maps must be current.
static hipError_t enqueue_hessian(cel_plan* p, const double* theta, const int32_t* order, int n_items,
                                  const int32_t* srcs, int n_src, const uint8_t* active, bool with_kl, double* local,
                                  double* grad, double* hess, hipStream_t sm) {
  const bool fp64 = p->opt.pixel_fp64 || p->opt.hessian_fp64;
  hipError_t e = fp64 ? launch_hess_t<double>(p, order, n_items, active, sm)
                      : launch_hess_t<float>(p, order, n_items, active, sm);
  if (e != hipSuccess || n_src <= 0) return e;
  HessFinArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.job_src = srcs;
  fa.n_jobs = n_src;
  fa.active = active;
  fa.theta = theta;
  fa.hslots = p->d_hslots;
  fa.patch_ptr = p->d_patch_ptr;
  fa.patches = p->d_patches;
  fa.pix_const = p->d_pixconst;
  fa.images = p->d_images;
  fa.prior = p->d_prior;
  fa.with_kl = with_kl ? 1 : 0;
  fa.local = local;
  fa.grad = grad;
  fa.hess = hess;
  fa.err = with_kl ? p->d_err : nullptr;   // the Newton path reports through the step status
  fa.part = p->d_hpart;
  hipLaunchKernelGGL(k_hess_finalize, dim3(n_src, kHParts), dim3(64), 0, sm, fa);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hess_combine, dim3(n_src), dim3(64), 0, sm, fa);
  return hipGetLastError();
}

// One Newton iteration of colour class `cls` on the sources flagged in `active`.  With
// maps_current the neighbour moment maps are taken as they are (none of the class's
// neighbours has moved since they were made: the sweep refreshes them once per class) and
// only the class's own tables are rebuilt.
static hipError_t enqueue_newton_class(cel_plan* p, double* theta, double* radius, uint8_t* active, int cls,
                                       int32_t* status, double* out_local, bool clear_done, hipStream_t sm,
                                       bool maps_current = false) {
  const bool fp64 = p->opt.pixel_fp64 || p->opt.hessian_fp64;
  const int nsrc = (int)p->class_src[cls].size();
  if (nsrc == 0) return hipSuccess;
  hipError_t e;
  const bool analytic = !p->opt.hessian_fd;
  if (analytic) {
    // tables (and maps) at the iterate, then the exact Hessians with the gradients
    e = maps_current ? prep_class(p, theta, cls, active, sm, fp64, true) : prep_base(p, theta, sm, fp64, true);
    if (e == hipSuccess)
      e = enqueue_hessian(p, theta, p->d_class_tasks[cls], (int)p->class_tasks[cls].size(), p->d_class_src[cls], nsrc,
                          active, true, p->v_local, p->v_grad, p->d_hess, sm);
  } else {
    // gradients at the iterate and at the 54 central-difference points, then the Hessians
    e = eval_any(p, theta, nullptr, 0, 2 * kParamN + 1, true, cls, active, sm, true, fp64);
    if (e == hipSuccess) {
      FdHessArgs fa;
      std::memset(&fa, 0, sizeof(fa));
      fa.job_src = p->d_class_src[cls];
      fa.n_jobs = nsrc;
      fa.S = p->S;
      fa.active = active;
      fa.v_grad = p->v_grad;
      fa.fd_step = p->opt.fd_step;
      fa.theta = theta;
      fa.prior = p->d_prior;
      fa.hess = p->d_hess;
      hipLaunchKernelGGL(k_fd_hessian, dim3(nsrc), dim3(64), 0, sm, fa);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return e;
  TrArgs ta;
  std::memset(&ta, 0, sizeof(ta));
  ta.job_src = p->d_class_src[cls];
  ta.n_jobs = nsrc;
  ta.active = active;
  ta.v_grad = p->v_grad;
  ta.v_local = p->v_local;
  ta.hess = p->d_hess;
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
  ta.err = p->d_err;
  hipLaunchKernelGGL(k_trsolve, dim3(nsrc), dim3(64), 0, sm, ta);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // objective at the trial points
  e = eval_any(p, theta, p->d_theta_trial, p->trial_variant, 1, false, cls, p->d_trial_active, sm, false, fp64);
  if (e != hipSuccess) return e;
  AcceptArgs aa;
  std::memset(&aa, 0, sizeof(aa));
  aa.job_src = p->d_class_src[cls];
  aa.n_jobs = nsrc;
  aa.active = active;
  aa.clear_done = clear_done ? 1 : 0;
  aa.trial_active = p->d_trial_active;
  aa.local0 = p->v_local;
  aa.local_trial = p->v_local + (int64_t)p->trial_variant * p->S;
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
  // analytic Hessian: variants 0 (iterate) and 1 (trial); differences: 0, 1..54, 55 (trial)
  p->fd_mode = p->opt.hessian_fd ? 1 : 0;
  p->trial_variant = p->opt.hessian_fd ? kVariants - 1 : 1;
  cel_status st = ensure_variants(p, p->trial_variant + 1, fp64);
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
  // The stepped sources never overlap one another, so none is a neighbour of another: the
  // tables and neighbour maps made once at the iterate serve all of them, and the sources
  // of several colour classes are stepped as one batch (the step class).
  std::vector<int> used;
  for (int c = 0; c < p->n_colours; ++c) {
    bool any = false;
    for (int s : p->class_src[c]) any = any || m[s];
    if (any) used.push_back(c);
  }
  int cls = used.empty() ? -1 : used[0];
  const bool union_class = used.size() > 1 && !p->opt.hessian_fd;
  if (union_class) cls = p->n_colours;
  hipError_t e = stage_selection(p, m, union_class, sm);
  const bool maps_once = !p->opt.hessian_fd;
  if (maps_once && e == hipSuccess && cls >= 0) e = prep_base(p, theta, sm, p->opt.pixel_fp64 || p->opt.hessian_fp64);
  if (cls == p->n_colours) {
    if (e == hipSuccess) e = enqueue_newton_class(p, theta, radius, p->d_mask, cls, step_status, elbo_local, false, sm, true);
  } else {
    for (int c : used) {
      if (e != hipSuccess) break;
      e = enqueue_newton_class(p, theta, radius, p->d_mask, c, step_status, elbo_local, false, sm, maps_once);
    }
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
  std::memset(&o, 0, sizeof(o));
  o.n_sweeps = 3;
  o.max_newton_iters = 50;
  o.use_graph = 1;
  if (opts) {
    if (opts->n_sweeps < 0 || opts->max_newton_iters < 0 || opts->max_classes < 0 || opts->start_colour < 0 ||
        (opts->start_colour > 0 && opts->start_colour >= cplan->n_colours))
      return CEL_EINVAL;
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
  if (S > 0 && o.start_colour == 0) {   // a fresh pass: every status starts as skipped
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
  int classes = 0, sweeps_done = 0, next_colour = 0;
  bool stopped = false;
  for (int sw = 0; sw < o.n_sweeps && e == hipSuccess && S > 0 && !stopped; ++sw) {
    const int c0 = sw == 0 ? o.start_colour : 0;
    if (c0 == 0) {   // trust radii restart at each pass
      hipLaunchKernelGGL(k_fill_radius, dim3((S + 255) / 256), dim3(256), 0, sm, radius, S, p->opt.radius0);
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    for (int c = c0; c < p->n_colours && e == hipSuccess; ++c) {
      if (o.max_classes > 0 && classes == o.max_classes) {
        stopped = true;
        next_colour = c;
        break;
      }
      ++classes;
      const int nsrc = (int)p->class_src[c].size();
      hipLaunchKernelGGL(k_set_active, dim3((S + 255) / 256), dim3(256), 0, sm, p->d_mask, p->d_colour, S, c);
      if ((e = hipGetLastError()) != hipSuccess) break;
      // the neighbours of this class keep their parameters during its iterations: their
      // moment maps are made once here (analytic Hessian path)
      const bool maps_once = !p->opt.hessian_fd;
      if (maps_once && (e = prep_base(p, theta, sm, p->opt.pixel_fp64 || p->opt.hessian_fp64)) != hipSuccess) break;
      hipGraphExec_t exec = nullptr;
      if (o.use_graph) {
        auto& G = p->graphs[c];
        if (!G.exec || G.theta != theta || G.radius != radius || G.status != status || G.stream != sm) {
          if (G.exec) (void)hipGraphExecDestroy(G.exec);
          G.exec = nullptr;
          hipGraph_t graph;
          e = hipStreamBeginCapture(sm, hipStreamCaptureModeThreadLocal);
          if (e != hipSuccess) break;
          hipError_t e2 = enqueue_newton_class(p, theta, radius, p->d_mask, c, status, nullptr, true, sm, maps_once);
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
        else e = enqueue_newton_class(p, theta, radius, p->d_mask, c, status, nullptr, true, sm, maps_once);
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
    if (!stopped && e == hipSuccess) ++sweeps_done;
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
    report->sweeps_done = sweeps_done;
    report->next_colour = next_colour;
  }
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}

extern "C" cel_status cel_elbo_hessian(cel_ctx* ctx, const cel_plan* cplan, const double* theta, const uint8_t* mask,
                                       double* hess, double* grad, double* elbo_local, void* stream) {
  if (!ctx || !cplan) return CEL_EINVAL;
  cel_plan* p = const_cast<cel_plan*>(cplan);
  if (p->S > 0 && (!theta || !hess)) return CEL_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return CEL_EHIP;
  hipStream_t sm = (hipStream_t)stream;
  cel_status st = newton_scratch(p);
  if (st) return st;
  if (p->S == 0) return CEL_OK;
  const bool fp64 = p->opt.pixel_fp64 || p->opt.hessian_fp64;
  if (hipEventSynchronize(p->mask_copied) != hipSuccess) return CEL_EHIP;
  for (int s = 0; s < p->S; ++s) p->h_mask[s] = mask ? (mask[s] ? 1 : 0) : 1;
  hipError_t e = hipMemcpyAsync(p->d_mask, p->h_mask, p->S, hipMemcpyHostToDevice, sm);
  if (e == hipSuccess) e = hipEventRecord(p->mask_copied, sm);
  if (e == hipSuccess) e = prep_base(p, theta, sm, fp64, true);
  if (e == hipSuccess)
    e = enqueue_hessian(p, theta, p->d_order, (int)p->n_tasks, nullptr, p->S, p->d_mask, true,
                        elbo_local ? elbo_local : p->v_local, grad ? grad : p->v_grad, hess, sm);
  return e == hipSuccess ? CEL_OK : CEL_EHIP;
}
