// Device helpers shared by the celmi kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "device.h"

namespace celmi {

// ----------------------------------------------------------------------------------------
// precision helpers

template <typename T> __device__ __forceinline__ T fexp2(T x);
template <> __device__ __forceinline__ float fexp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double fexp2<double>(double x) { return exp2(x); }

constexpr double kLn2 = 0.69314718055994530942;

// x log(E/x) for a count x > 0 and a rate E > 0: the part of the centred Poisson term that
// cancels against E - x, so the quotient must be accurate to the last bit or two.  float:
// the quotient from the hardware reciprocal with one residual correction (within an ulp of
// E/x for normal operands), the logarithm from the hardware log2 (operands here are
// normal: x >= 1, E at least the patch's smallest sky value); double: library division
// and logarithm.
template <typename T> __device__ __forceinline__ T x_log_ratio(T x, T E);
template <> __device__ __forceinline__ float x_log_ratio<float>(float x, float E) {
  const float r = __builtin_amdgcn_rcpf(x);
  float q = E * r;
  q = fmaf(fmaf(-x, q, E), r, q);
  return x * (__builtin_amdgcn_logf(q) * (float)kLn2);
}
template <> __device__ __forceinline__ double x_log_ratio<double>(double x, double E) { return x * log(E / x); }

// 1/E for the adjoint coefficients (float: hardware reciprocal, within 1 ulp)
template <typename T> __device__ __forceinline__ T frcp(T E);
template <> __device__ __forceinline__ float frcp<float>(float E) { return __builtin_amdgcn_rcpf(E); }
template <> __device__ __forceinline__ double frcp<double>(double E) { return 1.0 / E; }

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLog2TwoPi = 2.6514961294723187980;   // log2(2 pi)
constexpr double kNegHuge = -1.0e30;
// Block -> position in a cost-sorted work list, XCD-aware.  Workgroups are dispatched to
// the 8 XCDs in turn (block b on XCD b mod 8), each XCD with its own L2.  Consecutive
// positions of the list (the chunks of one patch, sorted next to each other) are handed to
// one XCD in groups of kXcdGroup, so they share its L2 (tables, neighbour maps); the list
// order across groups, and so the large-first balance, is kept.  A tail that does not fill
// whole groups maps to itself.
constexpr int kXcds = 8;
constexpr int kXcdGroup = 4;
__device__ __forceinline__ int xcd_position(int b, int n) {
  constexpr int span = kXcds * kXcdGroup;
  const int full = (n / span) * span;
  if (b >= full) return b;
  const int xcd = b % kXcds, slot = b / kXcds;
  return ((slot / kXcdGroup) * kXcds + xcd) * kXcdGroup + slot % kXcdGroup;
}

// Component cut (reading of the kernels' truncation): a mixture component is skipped over a
// wavefront's pixel box when its contribution to the expected count there, flux times
// density, stays below 2^-kRelCut of the patch's smallest sky value -- far below the
// resolution of the rate in the kernel's precision (2^-24 in float32, 2^-53 in float64).
template <typename T>
constexpr double rel_cut_log2() {
  return sizeof(T) == 8 ? 60.0 : 30.0;
}

// Value of one mixture component at offset (dx, dy) from its centre, given the monomials
// xx = dx^2, xy = 2 dx dy, yy = dy^2 and its record q = (q0, q1, q2, log2 weight):
// 2^(q0 xx + q1 xy + q2 yy + lw) -- the form for values alone (neighbour maps, Hessian);
// the pixel kernel, which needs u = P d for the derivatives anyway, forms the exponent
// from u (the same value up to rounding).
template <typename T>
__device__ __forceinline__ T comp_value(const T* __restrict__ q, T xx, T xy, T yy) {
  return fexp2<T>(fma(q[0], xx, fma(q[1], xy, fma(q[2], yy, q[3]))));
}


// squared radius beyond which 2^(lw - log2(e)/2 d^T C^{-1} d) < 2^cut (-1: never above it;
// +inf when the component is not finite, so that NaN parameters reach the rate)
__device__ __forceinline__ double cut_radius2(double lw, double cxx, double cxy, double cyy, double cut) {
  const double room = lw - cut;
  const double lmax = 0.5 * (cxx + cyy) + sqrt(0.25 * (cxx - cyy) * (cxx - cyy) + cxy * cxy);
  if (isnan(room) || !isfinite(lmax)) return INFINITY;
  if (!(room > 0)) return -1.0;
  return room * lmax * (2.0 / kLog2e);
}

// log2 threshold on a component's density for a source of expected flux L on a patch whose
// sky is at least sky_min; -inf (keep everything) when either is not a positive finite
// number, so that non-finite parameters still propagate to the objective
template <typename T>
__device__ __forceinline__ double density_cut_log2(double L, double sky_min, double log2_L, double log2_sky_min) {
  const double c = log2_sky_min - log2_L - rel_cut_log2<T>();
  return (L > 0 && sky_min > 0 && isfinite(c)) ? c : -INFINITY;
}

// log l_b = log r + W[b] . c,  c_k = ln(l_{k+1} / l_k), reference band r = index 2
static __device__ __constant__ double c_W[5][4] = {
    {-1, -1, 0, 0}, {0, -1, 0, 0}, {0, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 1, 1}};

__device__ __forceinline__ double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }
__device__ __forceinline__ double softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }



// Squared distance from (mx, my) to the wavefront's pixel box [bx0, bx1] x [by0, by1].
// The component cut compares a wavefront-uniform squared distance d2 (>= +0, possibly +inf)
// with a stored squared cut radius that is never -0 or NaN (the tables are written so).  For
// such values the order of IEEE floats is the signed order of their bit patterns, so the
// float path takes each test as an integer compare of scalar registers instead of one vector
// compare per component; the double path compares the values.
__device__ __forceinline__ int cut_key(float x) { return __float_as_int(x); }
__device__ __forceinline__ double cut_key(double x) { return x; }
__device__ __forceinline__ int uniform_cut_key(float d2) { return __builtin_amdgcn_readfirstlane(__float_as_int(d2)); }
__device__ __forceinline__ double uniform_cut_key(double d2) { return d2; }

template <typename T>
__device__ __forceinline__ T box_dist2(T mx, T my, const T* box) {
  const T ddx = fmax(fmax(box[0] - mx, mx - box[1]), (T)0);
  const T ddy = fmax(fmax(box[2] - my, my - box[3]), (T)0);
  return ddx * ddx + ddy * ddy;
}

// Pixel box (patch-local columns x0..x1, rows y0..y1) of the run [base, end) of a
// row-major patch of width w.
template <typename T>
__device__ __forceinline__ void run_box(int base, int end, int w, T* box) {
  const int last = end - 1;
  const int r0 = base / w, r1 = last / w;
  box[0] = (T)(r0 == r1 ? base - r0 * w : 0);
  box[1] = (T)(r0 == r1 ? last - r1 * w : w - 1);
  box[2] = (T)r0;
  box[3] = (T)r1;
}

template <typename T>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wavefront sums of M values per lane together.  At each lane offset O = 32, 16, ... a lane
// keeps half of its values (the first half when bit O of its index is clear, else the second)
// and adds the partner lane's copies of those, so the values per lane halve at every step
// (M/2 + M/4 + ... exchanges instead of 6 M); once one value is left a plain butterfly
// finishes.  Every sum takes the same additions, in the same pairing and operand order, as
// wave_sum's butterfly, so the results are bitwise those of M wave_sum calls.  U is the
// type the lanes hold (float values are exchanged as floats and widened before the first
// addition, which is exact).  Lane l returns the sum of value wave_sums_slot<M>(l) (-1: none;
// each value has exactly one such lane).
template <int M, int O = 32, typename U>
__device__ __forceinline__ double wave_sums(const U* v, int lane) {
  if constexpr (M == 1) {
    double x = (double)v[0];
#pragma unroll
    for (int off = O; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
  } else {
    static_assert(O >= 1, "more values than lanes");
    constexpr int A = (M + 1) / 2, B = M - A;
    const bool hi = (lane & O) != 0;
    double w[A];
#pragma unroll
    for (int i = 0; i < A; ++i) {
      const U f = v[i], s = i < B ? v[A + i] : (U)0;
      const U send = hi ? f : s;
      w[i] = (double)(hi ? s : f) + (double)__shfl_xor(send, O, 64);
    }
    return wave_sums<A, O / 2, double>(w, lane);
  }
}

// the lane that wave_sums leaves holding the sum of value q (the lowest such lane)
template <int M, int O = 32>
__host__ __device__ constexpr int wave_sums_lane(int q) {
  if constexpr (M == 1) {
    return 0;
  } else {
    constexpr int A = (M + 1) / 2;
    return q < A ? wave_sums_lane<A, O / 2>(q) : O + wave_sums_lane<A, O / 2>(q - A);
  }
}

// a double held by lane l, read by every lane (l wavefront-uniform)
__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

template <int M, int O = 32>
__device__ __forceinline__ int wave_sums_slot(int lane) {
  if constexpr (M == 1) {
    return (O == 0 || (lane & (2 * O - 1)) == 0) ? 0 : -1;
  } else {
    constexpr int A = (M + 1) / 2, B = M - A;
    const int r = wave_sums_slot<A, O / 2>(lane);
    if (r < 0) return -1;
    if (lane & O) return r < B ? A + r : -1;
    return r;
  }
}

// Colour bounds of both types (Section 4.2.3 at their optimal weights): the values
// -log sum_j w_j exp(-D_j) and their gradients with respect to the colour means (gm) and
// log colour variances (gv), summed over the prior components j with weights xi_j,
// computed by a whole wavefront (all 64 lanes active): lane 8 i + j
// takes prior component j of type i (lanes 16..63 repeat lanes 0..15), the maximum,
// normaliser and gradient sums are combined by fixed butterflies within each group of 8
// lanes, and every lane receives both types' results.
__device__ inline void colour_bound_wave(const DPrior& pr, const double* th, int lane, double* kc, double (*gm)[4],
                                         double (*gv)[4]) {
  static_assert(CEL_N_COLOUR_COMPONENTS == 8, "one lane per prior colour component, groups of 8");
  const int i = (lane >> 3) & 1, j = lane & 7;
  double cm[4], cv[4], lcv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {   // selects, not a lane-dependent index into th
    cm[k] = i ? th[11 + k] : th[7 + k];
    lcv[k] = i ? th[19 + k] : th[15 + k];
    cv[k] = exp(lcv[k]);
  }
  const double sum_lcv = lcv[0] + lcv[1] + lcv[2] + lcv[3];
  double tr = 0, maha = 0, row[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    tr += pr.c_prec[i][j][k][k] * cv[k];
    double r = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) r += pr.c_prec[i][j][k][l] * (cm[l] - pr.c_mean[i][j][l]);
    row[k] = r;
    maha += (cm[k] - pr.c_mean[i][j][k]) * r;
  }
  const double e = pr.c_logw[i][j] - 0.5 * (tr + maha - 4.0 + pr.c_logdet[i][j] - sum_lcv);
  double mx = e;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const double ex = exp(e - mx);
  double z = ex;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) z += __shfl_xor(z, off, 64);
  const double xi = ex / z;
  double part[9];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    part[k] = xi * row[k];
    part[4 + k] = xi * 0.5 * (pr.c_prec[i][j][k][k] * cv[k] - 1.0);
  }
  part[8] = -(mx + log(z));
#pragma unroll
  for (int q = 0; q < 8; ++q) {
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) part[q] += __shfl_xor(part[q], off, 64);
  }
  // this lane's group holds type i; the other type comes from the group 8 lanes away
  double other[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) other[q] = __shfl_xor(part[q], 8, 64);
  const bool first = i == 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    gm[0][k] = first ? part[k] : other[k];
    gm[1][k] = first ? other[k] : part[k];
    gv[0][k] = first ? part[4 + k] : other[4 + k];
    gv[1][k] = first ? other[4 + k] : part[4 + k];
  }
  kc[0] = first ? part[8] : other[8];
  kc[1] = first ? other[8] : part[8];
}

// KL(q(z_s) || p(z_s)) and its gradient in the unconstrained coordinates (equations eq:kl,
// kleq; Supplement A with the readings: flux KL is the normal KL of log r with variances;
// colour KL is the bound of Section 4.2.3 at its optimal weights; point-mass terms are
// minus the log prior density; direction and angle terms are constants and dropped), given
// the colour bounds kc and their gradients.  Subtracts gs times the gradient from g.
__device__ inline double kl_assemble(const DPrior& pr, const double* th, double* g, double gs, const double* kc,
                                     const double (*gm)[4], const double (*gv)[4]) {
  const double eta = th[2];
  const double a = sigmoid(eta);
  const double log_a = -softplus(-eta), log_1ma = -softplus(eta);
  double kl = a * (log_a - pr.log_a) + (1.0 - a) * (log_1ma - pr.log_1ma);
  double dk_da = eta - pr.logit_a;          // d KL_a / d a
  const double q[2] = {1.0 - a, a};
  double part[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double rm = th[3 + i], lrv = th[5 + i], rv = exp(lrv);
    const double R1 = pr.r[i][0], R2 = pr.r[i][1];
    const double kr = 0.5 * (log(R2) - lrv) + (rv + (rm - R1) * (rm - R1)) / (2.0 * R2) - 0.5;
    g[3 + i] -= gs * q[i] * (rm - R1) / R2;
    g[5 + i] -= gs * q[i] * (-0.5 + rv / (2.0 * R2));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      g[7 + 4 * i + k] -= gs * q[i] * gm[i][k];
      g[15 + 4 * i + k] -= gs * q[i] * gv[i][k];
    }
    part[i] = kr + kc[i];
    kl += q[i] * part[i];
  }
  dk_da += part[1] - part[0];
  g[2] -= gs * (dk_da * a * (1.0 - a));
  // radius: point mass vs log-normal
  const double lr = th[24], E1 = pr.radius[0], E2 = pr.radius[1];
  kl += lr + 0.5 * log(2.0 * M_PI * E2) + (lr - E1) * (lr - E1) / (2.0 * E2);
  g[24] -= gs * (1.0 + (lr - E1) / E2);
  // profile and axis: point mass vs Beta
  {
    const double e = th[25], p = sigmoid(e), lp = -softplus(-e), l1p = -softplus(e);
    kl += -(pr.profile[0] - 1.0) * lp - (pr.profile[1] - 1.0) * l1p + pr.lbeta_profile;
    g[25] -= gs * (-(pr.profile[0] - 1.0) * (1.0 - p) + (pr.profile[1] - 1.0) * p);
  }
  {
    const double e = th[26], p = sigmoid(e), lp = -softplus(-e), l1p = -softplus(e);
    kl += -(pr.axis[0] - 1.0) * lp - (pr.axis[1] - 1.0) * l1p + pr.lbeta_axis;
    g[26] -= gs * (-(pr.axis[0] - 1.0) * (1.0 - p) + (pr.axis[1] - 1.0) * p);
  }
  return kl;
}

// KL and gradient by a whole wavefront (all lanes active; every lane gets the value and
// applies the gradient to its own g)
__device__ inline double kl_source_wave(const DPrior& pr, const double* th, double* g, double gs, int lane) {
  double kc[2], gm[2][4], gv[2][4];
  colour_bound_wave(pr, th, lane, kc, gm, gv);
  return kl_assemble(pr, th, g, gs, kc, gm, gv);
}

}  // namespace celmi
