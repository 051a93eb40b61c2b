// kernels.hip -- the reductions (stable time step, integrals, finiteness)
// and the dispatch of the DGSEM kernels over the polynomial degree.  The
// kernels of the time derivative are templates in kernels.h, instantiated
// per degree in kernels_n<N>.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dg_internal.h"
#include "physics.h"

namespace dg {

// ---------------------------------------------------------------------------
// reductions (per-block partials; the host finishes them)
// ---------------------------------------------------------------------------
template <int N, typename real>
__global__ void __launch_bounds__(256) k_dt(View<real> v, double *out) {
  constexpr int n = N + 1, n3 = n * n * n;
  __shared__ double s0[256], s1[256];
  const int64_t tot = v.E * n3;
  double dta = 1e300, dtv = 1e300;
  const double gam = (double)v.gamma;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
    const int64_t e = t / n3;
    const int a = (int)(t - e * n3);
    double U[5], P[6];
#pragma unroll
    for (int c = 0; c < 5; ++c) U[c] = v.U[((int64_t)c * v.E + e) * n3 + a];
    cons2prim(U, gam, (double)v.rRgas, P);
    const double c = sqrt(gam * P[4] / P[0]);
    const double iJ = (double)v.invJ[e * n3 + a];
    double lamsum = 0.0, vis = 0.0;
#pragma unroll
    for (int ci = 0; ci < 3; ++ci) {
      const double j0 = v.Ja[((int64_t)(3 * ci) * v.E + e) * n3 + a];
      const double j1 = v.Ja[((int64_t)(3 * ci + 1) * v.E + e) * n3 + a];
      const double j2 = v.Ja[((int64_t)(3 * ci + 2) * v.E + e) * n3 + a];
      const double nj = sqrt(j0 * j0 + j1 * j1 + j2 * j2);
      lamsum += (fabs(P[1] * j0 + P[2] * j1 + P[3] * j2) + c * nj) * iJ;
      vis += (nj * iJ) * (nj * iJ);
    }
    dta = fmin(dta, 2.0 / ((2.0 * N + 1.0) * lamsum));
    if (v.viscous && v.mu > 0) {
      const double mun = v.visc_law ? sutherland<double>(P[5], (double)v.mu, (double)v.rTref) : (double)v.mu;
      const double nu = fmax(4.0 / 3.0, gam / v.Pr) * mun / P[0];
      dtv = fmin(dtv, 4.0 / (pow((double)n, 4.0) * nu * vis));
    }
  }
  s0[threadIdx.x] = dta;
  s1[threadIdx.x] = dtv;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + w]);
      s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = s0[0];
    out[2 * blockIdx.x + 1] = s1[0];
  }
}

template <int N, typename real>
__global__ void __launch_bounds__(256) k_integrals(View<real> v, double *out) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  __shared__ double sw[n];
  __shared__ double s[7][256];
  BasisOffsets o(n);
  for (int t = threadIdx.x; t < n; t += 256) sw[t] = (double)v.basis[o.w + t];
  __syncthreads();
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t tot = v.E * n3;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
    const int64_t e = t / n3;
    const int a = (int)(t - e * n3);
    const int i = a % n, j = (a / n) % n, k = a / n2;
    const double wJ = sw[i] * sw[j] * sw[k] / (double)v.invJ[e * n3 + a];
    double U[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U[c] = v.U[((int64_t)c * v.E + e) * n3 + a];
      acc[c] += wJ * U[c];
    }
    acc[5] += wJ * 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
    acc[6] += wJ;
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) s[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < 7; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) out[7 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_finite(const double *U, int64_t count, int *flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256)
    if (!isfinite(U[t])) mine = 1;
  if (mine) bad = 1;  // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(flag, 1);
}

// sums of the per-element triples in[3 e + c] over e < E into out[0..2], in a
// fixed order (one workgroup: strided partial sums per thread, then a tree),
// so the result does not depend on the launch
__global__ void __launch_bounds__(1024) k_sum3(const double *in, int64_t E, double *out) {
  __shared__ double s[3][1024];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t e = threadIdx.x; e < E; e += 1024) {
    a0 += in[3 * e];
    a1 += in[3 * e + 1];
    a2 += in[3 * e + 2];
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  s[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_zero_int(int *p, int count) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < count; t += gridDim.x * 256) p[t] = 0;
}

__global__ void __launch_bounds__(256) k_cast(const double *src, float *dst, int64_t count) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256)
    dst[t] = (float)src[t];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
static int blocks_for(int64_t E) {
  return (int)((E + Sz<N>::epb - 1) / Sz<N>::epb);
}

#define DG_FOR_N(MACRO) \
  MACRO(1) MACRO(2) MACRO(3) MACRO(4) MACRO(5) MACRO(6) MACRO(7) MACRO(8) MACRO(9)

int blocks_per_elements(int N, int64_t E) {
  switch (N) {
#define CASE(NN) \
  case NN: return blocks_for<NN>(E);
    DG_FOR_N(CASE)
#undef CASE
  }
  return 0;
}

int block_threads(int N) {
  switch (N) {
#define CASE(NN) \
  case NN: return Sz<NN>::threads;
    DG_FOR_N(CASE)
#undef CASE
  }
  return 0;
}

template <typename real>
hipError_t launch(Kernel k, int N, int mode, const View<real> *views_dev, const int *blk_start_dev, int nreq,
                  int total_blocks, const View<real> &v0, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  switch (N) {
#define CASE(NN) \
  case NN: return launch_n<NN, real>(k, mode, views_dev, blk_start_dev, nreq, total_blocks, v0, st);
    DG_FOR_N(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <typename real>
hipError_t launch_dt(int N, const View<real> &v, double *scratch, int nblk, hipStream_t st) {
  switch (N) {
#define CASE(NN) \
  case NN: k_dt<NN, real><<<nblk, 256, 0, st>>>(v, scratch); return hipGetLastError();
    DG_FOR_N(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <typename real>
hipError_t launch_integrals(int N, const View<real> &v, double *scratch, int nblk, hipStream_t st) {
  switch (N) {
#define CASE(NN) \
  case NN: k_integrals<NN, real><<<nblk, 256, 0, st>>>(v, scratch); return hipGetLastError();
    DG_FOR_N(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finite(const double *U, int64_t count, int *flag, hipStream_t st) {
  k_finite<<<256, 256, 0, st>>>(U, count, flag);
  return hipGetLastError();
}

hipError_t launch_sum3(const double *in, int64_t E, double *out, hipStream_t st) {
  k_sum3<<<1, 1024, 0, st>>>(in, E, out);
  return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int count, hipStream_t st) {
  k_zero_int<<<std::max(1, std::min(64, (count + 255) / 256)), 256, 0, st>>>(p, count);
  return hipGetLastError();
}

hipError_t launch_cast(const double *src, float *dst, int64_t count, hipStream_t st) {
  int nb = (int)std::min<int64_t>(4096, (count + 255) / 256);
  if (nb < 1) nb = 1;
  k_cast<<<nb, 256, 0, st>>>(src, dst, count);
  return hipGetLastError();
}

template hipError_t launch<double>(Kernel, int, int, const View<double> *, const int *, int, int, const View<double> &,
                                   hipStream_t);
template hipError_t launch<float>(Kernel, int, int, const View<float> *, const int *, int, int, const View<float> &,
                                  hipStream_t);
template hipError_t launch_dt<double>(int, const View<double> &, double *, int, hipStream_t);
template hipError_t launch_dt<float>(int, const View<float> &, double *, int, hipStream_t);
template hipError_t launch_integrals<double>(int, const View<double> &, double *, int, hipStream_t);
template hipError_t launch_integrals<float>(int, const View<float> &, double *, int, hipStream_t);

}  // namespace dg
