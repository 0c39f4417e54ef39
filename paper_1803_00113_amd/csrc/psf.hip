// Spatially varying PSF (gfx950): reconstruction of an image's PSF at a position from its
// eigen-images and the fit of a Gaussian mixture to it (Section 2.2.2, Table 1: E principal
// images on a side x side grid centred on a source, loadings varying smoothly over the
// image; Section 2.2.3: the PSF approximated by a mixture of bivariate normals).
//
// k_psf_fit: one workgroup of 256 threads per fit, all arithmetic in FP64.  The PSF image
// (at most 63 x 63 knots) is formed once in LDS; each expectation-maximisation iteration
// evaluates the K component densities at every knot, accumulates per component the weighted
// sums of 1, dx, dy, dx^2, dx dy, dy^2 over the responsibilities, reduces them across the
// workgroup in a fixed order (wavefront butterflies, then the four wavefronts in order) and
// forms the next mixture.  Deterministic: no atomics.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cstring>

#include "device.h"
#include "plan.h"

namespace celmi {

constexpr int kPsfThreads = 256;
constexpr int kPsfWaves = kPsfThreads / kWave;
constexpr int kPsfMaxSide = CEL_PSF_MAX_SIDE;
constexpr int kPsfSums = 6 * kMaxPsf;

struct PsfFitArgs {
  int32_t n_images, n_eigen, side;
  const double* eigen;      // [n_images][n_eigen][side][side]
  const double* coef;       // [n_images][n_eigen][6]
  const double* size;       // [n_images][2]: W, H
  const int32_t* fit_img;   // [n]
  const double* fit_xy;     // [n][2]
  int32_t K, n_iter;
  double* out;              // [n][kMaxPsf][6]
  int32_t* err;
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum each of the L per-thread values over the workgroup (fixed order) into red_out[0..L).
template <int L>
__device__ __forceinline__ void block_sum(double (&v)[L], double (*red)[L], double* red_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < L; ++i) v[i] = wave_sum_d(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < L; ++i) red[wv][i] = v[i];
  __syncthreads();
  if ((int)threadIdx.x < L) {
    double s = 0.0;
    for (int w = 0; w < kPsfWaves; ++w) s += red[w][threadIdx.x];
    red_out[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double normal_density(double dx, double dy, const double* m) {
  // m: weight, mean x, mean y, cov xx, cov xy, cov yy
  const double det = m[3] * m[5] - m[4] * m[4];
  const double ex = dx - m[1], ey = dy - m[2];
  const double q = (m[5] * ex * ex - 2.0 * m[4] * ex * ey + m[3] * ey * ey) / det;
  return exp(-0.5 * q) / (2.0 * M_PI * sqrt(det));
}

__global__ __launch_bounds__(kPsfThreads) void k_psf_fit(PsfFitArgs a) {
  __shared__ double wts[kPsfMaxSide * kPsfMaxSide];
  __shared__ double red[kPsfWaves][kPsfSums];
  __shared__ double sums[kPsfSums];
  __shared__ double mix[kMaxPsf][6];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = a.fit_img[f];
  double* out = a.out + (int64_t)f * kMaxPsf * 6;
  if (n < 0 || n >= a.n_images) {   // a bad image index: this fit's rows are NaN
    if (tid < kMaxPsf * 6) out[tid] = NAN;
    if (tid == 0 && a.err) atomicOr(a.err, CEL_DEVERR_BAD_INDEX);
    return;
  }
  const int side = a.side, npx = side * side, E = a.n_eigen, K = a.K;
  const double c = 0.5 * (side - 1);
  // loadings at the fit position: quadratic in u = x / W, v = y / H
  const double u = a.fit_xy[2 * f] / a.size[2 * n], v = a.fit_xy[2 * f + 1] / a.size[2 * n + 1];
  const double mono[6] = {1.0, u, v, u * u, u * v, v * v};
  double load[kMaxPsf];
#pragma unroll
  for (int e = 0; e < kMaxPsf; ++e) {
    double s = 0.0;
    if (e < E)
#pragma unroll
      for (int t = 0; t < 6; ++t) s += a.coef[((int64_t)n * E + e) * 6 + t] * mono[t];
    load[e] = s;
  }
  // the PSF image, negative values clipped; its mass and centroid
  const double* eig = a.eigen + (int64_t)n * E * npx;
  double m3[kPsfSums];
#pragma unroll
  for (int i = 0; i < kPsfSums; ++i) m3[i] = 0.0;
  for (int p = tid; p < npx; p += kPsfThreads) {
    double s = 0.0;
    for (int e = 0; e < E; ++e) s += load[e] * eig[(int64_t)e * npx + p];
    s = s > 0.0 ? s : 0.0;
    wts[p] = s;
    const int i = p / side, j = p - (p / side) * side;
    const double dx = j - c, dy = i - c;
    m3[0] += s;
    m3[1] += s * dx;
    m3[2] += s * dy;
  }
  block_sum<kPsfSums>(m3, red, sums);
  const double M = sums[0], mx = sums[1] / M, my = sums[2] / M;
  __syncthreads();
  // central second moments (a second pass, about the centroid)
#pragma unroll
  for (int i = 0; i < kPsfSums; ++i) m3[i] = 0.0;
  for (int p = tid; p < npx; p += kPsfThreads) {
    const int i = p / side, j = p - (p / side) * side;
    const double dx = j - c - mx, dy = i - c - my, s = wts[p];
    m3[0] += s * dx * dx;
    m3[1] += s * dx * dy;
    m3[2] += s * dy * dy;
  }
  block_sum<kPsfSums>(m3, red, sums);
  if (tid < K) {   // the start: every component at the centroid, covariance scaled by 2^(k - (K-1)/2)
    const double fac = exp2((double)tid - 0.5 * (K - 1));
    mix[tid][0] = 1.0 / K;
    mix[tid][1] = mx;
    mix[tid][2] = my;
    mix[tid][3] = fac * sums[0] / M;
    mix[tid][4] = fac * sums[1] / M;
    mix[tid][5] = fac * sums[2] / M;
  }
  __syncthreads();
  for (int it = 0; it < a.n_iter; ++it) {
    double acc[kPsfSums];
#pragma unroll
    for (int i = 0; i < kPsfSums; ++i) acc[i] = 0.0;
    for (int p = tid; p < npx; p += kPsfThreads) {
      const double s = wts[p];
      if (s == 0.0) continue;
      const int i = p / side, j = p - (p / side) * side;
      const double dx = j - c, dy = i - c;
      double comp[kMaxPsf], tot = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxPsf; ++k) {
        comp[k] = k < K ? mix[k][0] * normal_density(dx, dy, mix[k]) : 0.0;
        tot += comp[k];
      }
      if (!(tot > 0.0)) continue;
      const double it_ = 1.0 / tot;
#pragma unroll
      for (int k = 0; k < kMaxPsf; ++k) {
        const double r = s * comp[k] * it_;
        acc[6 * k + 0] += r;
        acc[6 * k + 1] += r * dx;
        acc[6 * k + 2] += r * dy;
        acc[6 * k + 3] += r * dx * dx;
        acc[6 * k + 4] += r * dx * dy;
        acc[6 * k + 5] += r * dy * dy;
      }
    }
    block_sum<kPsfSums>(acc, red, sums);
    if (tid < K) {
      const double nk = sums[6 * tid];
      if (nk > 1e-12 * M) {   // a component with no weight keeps its parameters
        const double ax = sums[6 * tid + 1] / nk, ay = sums[6 * tid + 2] / nk;
        mix[tid][0] = nk / M;
        mix[tid][1] = ax;
        mix[tid][2] = ay;
        mix[tid][3] = sums[6 * tid + 3] / nk - ax * ax;
        mix[tid][4] = sums[6 * tid + 4] / nk - ax * ay;
        mix[tid][5] = sums[6 * tid + 5] / nk - ay * ay;
      }
    }
    __syncthreads();
  }
  // weights normalised to one; rows beyond K zero
  if (tid < kMaxPsf * 6) {
    const int k = tid / 6, q = tid - 6 * (tid / 6);
    double wsum = 0.0;
    for (int j = 0; j < K; ++j) wsum += mix[j][0];
    double val = 0.0;
    if (k < K) val = q == 0 ? mix[k][0] / wsum : mix[k][q];
    out[tid] = val;
  }
}

}  // namespace celmi

using namespace celmi;

extern "C" cel_status cel_psf_fit(cel_ctx* ctx, const cel_psf_model* model, int32_t n_fits, const int32_t* fit_img,
                                  const double* fit_xy, int32_t n_comp, int32_t n_iter, double* out, void* stream) {
  if (!ctx || !model || n_fits < 0 || n_comp < 1 || n_iter < 0 || n_iter > 100000) return CEL_EINVAL;
  if (n_comp > kMaxPsf || model->n_eigen > CEL_MAX_EIGEN || model->side > kPsfMaxSide) return CEL_EUNSUPPORTED;
  if (model->n_images < 0 || model->n_eigen < 1 || model->side < 3 || model->side % 2 == 0) return CEL_EINVAL;
  if (n_fits == 0) return CEL_OK;
  if (!fit_img || !fit_xy || !out || !model->eigen || !model->coef || !model->size || model->n_images < 1)
    return CEL_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return CEL_EHIP;
  PsfFitArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n_images = model->n_images;
  a.n_eigen = model->n_eigen;
  a.side = model->side;
  a.eigen = model->eigen;
  a.coef = model->coef;
  a.size = model->size;
  a.fit_img = fit_img;
  a.fit_xy = fit_xy;
  a.K = n_comp;
  a.n_iter = n_iter;
  a.out = out;
  a.err = ctx->d_err;
  hipLaunchKernelGGL(k_psf_fit, dim3(n_fits), dim3(kPsfThreads), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? CEL_OK : CEL_EHIP;
}
