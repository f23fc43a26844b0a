// Generic device kernels of libfsi: exclusive scan, CSR/BSR2 sparse products with fused
// epilogues (residual, Chebyshev step, prolongation-add), vector updates and
// deterministic reductions (fixed partition, fixed summation order, no float atomics).
#pragma once

#include "common.h"

namespace fsi {
// Everything here has internal linkage: each translation unit instantiates what it uses.
namespace {

// ------------------------------------------------------------------ exclusive scan
// out[i] = sum_{k<i} in[i] for i in [0, n]; out[n] is the total.  Three phases over
// tiles of 1024 items (256 threads x 4).
constexpr int kScanBlock = 256;
constexpr int kScanTile = 1024;

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one int per thread (256 threads); returns the block total.
__device__ __forceinline__ int block_excl_scan(int v, int &total) {
  __shared__ int wsum[kScanBlock / kWave];
  int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  int inc = wave_incl_scan(v, lane);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < kScanBlock / kWave; ++k) {
    if (k < w) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

__global__ void k_scan_sums(const int *in, int64_t n, int *bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + threadIdx.x * 4 + k;
    if (i < n) s += in[i];
  }
  int total;
  block_excl_scan(s, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void k_scan_bsums(int *bsum, int nb) {
  int carry = 0;
  for (int base = 0; base < nb; base += kScanBlock) {
    int i = base + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    int total;
    int ex = block_excl_scan(v, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void k_scan_final(const int *in, int64_t n, const int *bsum, int *out) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int v[4];
  int s = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + threadIdx.x * 4 + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int total;
  int ex = block_excl_scan(s, total) + bsum[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + threadIdx.x * 4 + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = bsum[gridDim.x];
}

// Tile sums a scan of n items needs (scan_tmp_len(n) ints of work space).
inline int64_t scan_tmp_len(int64_t n) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (nb < 1 ? 1 : nb) + 1;
}

// `in` and `out` may alias.  `tmp` holds the tile sums (at least scan_tmp_len(n) ints).
// Returns nothing: the total is out[n] on the device.
inline void scan_excl(const int *in, int *out, int64_t n, int *tmp, hipStream_t s) {
  const int nb = (int)(scan_tmp_len(n) - 1);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kScanBlock), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanBlock), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanBlock), 0, s, in, n, tmp, out);
  FSI_CHECK_LAUNCH();
}
inline void scan_excl(const int *in, int *out, int64_t n, DevBuf<int> &tmp, hipStream_t s) {
  tmp.reserve(scan_tmp_len(n));
  scan_excl(in, out, n, tmp.p, s);
}

// ------------------------------------------------------------------ sparse products
enum SpmvMode { SP_APPLY = 0, SP_RESID = 1, SP_ADD = 2, SP_CHEB = 3, SP_A11 = 4 };

// G lanes per row.  W = 4: 2x2 blocks on NC = 2 components; W = 1: the scalar matrix
// is applied to each of NC components.  Component c of a vector lives at v + c * stride.
//   SP_APPLY: y = A x
//   SP_RESID: y = b - A x
//   SP_ADD:   y = y + A x
//   SP_CHEB:  d = c1 d + c2 Dinv (b - A x);  y = x + d       (one Chebyshev step)
template <typename T, int W, int NC, int G, int MODE>
__global__ void __launch_bounds__(256) k_spmv(int64_t nrows, const int *__restrict__ rowptr,
                                              const int *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ x,
                                              int64_t xs, T *__restrict__ y, int64_t ys,
                                              const T *__restrict__ b, T *__restrict__ d,
                                              const T *__restrict__ dinv, T c1, T c2) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t row = gid / G;
  int lane = (int)(gid % G);
  if (row >= nrows) return;
  T s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = T(0);
  int k0 = rowptr[row], k1 = rowptr[row + 1];
  for (int k = k0 + lane; k < k1; k += G) {
    int j = col[k];
    if constexpr (W == 4) {
      T a00 = val[4 * (int64_t)k], a01 = val[4 * (int64_t)k + 1];
      T a10 = val[4 * (int64_t)k + 2], a11 = val[4 * (int64_t)k + 3];
      T x0 = x[j], x1 = x[xs + j];
      s[0] += a00 * x0 + a01 * x1;
      s[1] += a10 * x0 + a11 * x1;
    } else {
      T a = val[k];
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += a * x[c * xs + j];
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = group_sum<G>(s[c]);
  if (lane != 0) return;
  if constexpr (MODE == SP_APPLY) {
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c * ys + row] = s[c];
  } else if constexpr (MODE == SP_RESID) {
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c * ys + row] = b[c * ys + row] - s[c];
  } else if constexpr (MODE == SP_ADD) {
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c * ys + row] += s[c];
  } else {
    T r[NC], z[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c] = b[c * ys + row] - s[c];
    if constexpr (W == 4) {
      z[0] = dinv[4 * row] * r[0] + dinv[4 * row + 1] * r[1];
      z[1] = dinv[4 * row + 2] * r[0] + dinv[4 * row + 3] * r[1];
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) z[c] = dinv[row] * r[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T dn = c1 * d[c * ys + row] + c2 * z[c];
      d[c * ys + row] = dn;
      y[c * ys + row] = x[c * xs + row] + dn;
    }
  }
}

template <typename T, int W, int NC, int MODE>
inline void spmv(const int64_t nrows, const int *rowptr, const int *col, const T *val,
                 const T *x, int64_t xs, T *y, int64_t ys, hipStream_t s,
                 const T *b = nullptr, T *d = nullptr, const T *dinv = nullptr, T c1 = 0, T c2 = 0) {
  constexpr int G = (W == 4) ? 4 : 8;
  const int block = 256;
  unsigned grid = grid_for(nrows * G, block);
  hipLaunchKernelGGL((k_spmv<T, W, NC, G, MODE>), dim3(grid), dim3(block), 0, s, nrows, rowptr,
                     col, val, x, xs, y, ys, b, d, dinv, c1, c2);
  FSI_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ vector kernels
// The vector kernels below run over gridDim.y systems (lane = blockIdx.y, see LP).
template <typename T>
__global__ void k_fill(LP<T> xl, int64_t n, T v) {
  T *x = xl.at(blockIdx.y);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

template <typename To, typename Ti>
__global__ void k_convert(LP<To> yl, LP<const Ti> xl, int64_t n) {
  To *y = yl.at(blockIdx.y);
  const Ti *x = xl.at(blockIdx.y);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (To)x[i];
}

// y = a x + b y
template <typename T>
__global__ void k_axpby(T *y, const T *x, T a, T b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// z = a x + b y
template <typename TZ, typename T>
__global__ void k_lincomb(LP<TZ> zl, LP<const T> xl, LP<const T> yl, T a, T b, int64_t n) {   // z = a x + b y
  TZ *z = zl.at(blockIdx.y);
  const T *x = xl.at(blockIdx.y), *y = yl.at(blockIdx.y);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    z[i] = (TZ)(a * x[i] + b * y[i]);
}

inline unsigned vgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
inline void fill_l(LP<T> x, int64_t n, T v, hipStream_t s, int K) {
  hipLaunchKernelGGL(k_fill<T>, dim3(vgrid(n), K), dim3(256), 0, s, x, n, v);
  FSI_CHECK_LAUNCH();
}
template <typename T>
inline void fill(T *x, int64_t n, T v, hipStream_t s) {
  fill_l(LP<T>(x), n, v, s, 1);
}
template <typename To, typename Ti>
inline void convert_l(LP<To> y, LP<const Ti> x, int64_t n, hipStream_t s, int K) {
  hipLaunchKernelGGL((k_convert<To, Ti>), dim3(vgrid(n), K), dim3(256), 0, s, y, x, n);
  FSI_CHECK_LAUNCH();
}
template <typename To, typename Ti>
inline void convert(To *y, const Ti *x, int64_t n, hipStream_t s) {
  convert_l(LP<To>(y), LP<const Ti>(x), n, s, 1);
}
template <typename T>
inline void axpby(T *y, const T *x, T a, T b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(vgrid(n)), dim3(256), 0, s, y, x, a, b, n);
  FSI_CHECK_LAUNCH();
}
template <typename T>
inline void lincomb_l(LP<T> z, LP<const T> x, LP<const T> y, T a, T b, int64_t n, hipStream_t s, int K) {
  hipLaunchKernelGGL((k_lincomb<T, T>), dim3(vgrid(n), K), dim3(256), 0, s, z, x, y, a, b, n);
  FSI_CHECK_LAUNCH();
}
// z = a x + b y computed in T, stored as TZ
template <typename TZ, typename T>
inline void lincomb_to(TZ *z, const T *x, const T *y, T a, T b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_lincomb<TZ, T>), dim3(vgrid(n)), dim3(256), 0, s, LP<TZ>(z), LP<const T>(x), LP<const T>(y), a,
                     b, n);
  FSI_CHECK_LAUNCH();
}
template <typename T>
inline void lincomb(T *z, const T *x, const T *y, T a, T b, int64_t n, hipStream_t s) {
  lincomb_l(LP<T>(z), LP<const T>(x), LP<const T>(y), a, b, n, s, 1);
}

// ------------------------------------------------------------------ reductions
// Multi-dot: out[i] = sum_e V_i[e] * w[e] for i < k, V_i = V + i * ldv.  Accumulates in
// FP64.  Fixed partition into `nb` chunks (a function of n only) and fixed order.
constexpr int kRedBlock = 256;

inline int red_blocks(int64_t n) {
  int64_t nb = (n + 4095) / 4096;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double ws[kRedBlock / kWave];
  v = wave_sum(v);
  int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kRedBlock / kWave; ++k) t += ws[k];
  __syncthreads();
  return t;   // valid in thread 0
}

template <typename TV, typename TW>
__global__ void __launch_bounds__(kRedBlock) k_multidot_part(LP<const TV> Vl, int64_t ldv, int k,
                                                             LP<const TW> wl, int64_t n,
                                                             LP<double> partl) {
  const TV *V = Vl.at(blockIdx.y);
  const TW *w = wl.at(blockIdx.y);
  double *part = partl.at(blockIdx.y);
  int nb = gridDim.x;
  int64_t chunk = (n + nb - 1) / nb;
  int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk;
  if (hi > n) hi = n;
  for (int i = 0; i < k; ++i) {
    const TV *v = V + (int64_t)i * ldv;
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kRedBlock) s += (double)v[e] * (double)w[e];
    double t = block_sum(s);
    if (threadIdx.x == 0) part[(int64_t)i * nb + blockIdx.x] = t;
  }
}

// out[i] = sum_b part[i * nb + b] (one wavefront per i, fixed order)
__global__ void k_multidot_final(LP<const double> partl, int nb, int k, LP<double> outl) {
  const double *part = partl.at(blockIdx.y);
  double *out = outl.at(blockIdx.y);
  int i = blockIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kWave) s += part[(int64_t)i * nb + b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[i] = s;
}

template <typename TV, typename TW>
inline void multidot(const TV *V, int64_t ldv, int k, const TW *w, int64_t n, double *out,
                     DevBuf<double> &part, hipStream_t s) {
  int nb = red_blocks(n);
  part.reserve((size_t)nb * (k > 0 ? k : 1));
  hipLaunchKernelGGL((k_multidot_part<TV, TW>), dim3(nb), dim3(kRedBlock), 0, s, LP<const TV>(V), ldv, k,
                     LP<const TW>(w), n, LP<double>(part.p));
  hipLaunchKernelGGL(k_multidot_final, dim3(k), dim3(kWave), 0, s, LP<const double>(part.p), nb, k,
                     LP<double>(out));
  FSI_CHECK_LAUNCH();
}

// One dot product per lane (k = 1): out[lane] (lane stride of out) = V[lane] . w[lane];
// part holds red_blocks(n) partials per lane (lane stride red_blocks(n)), allocated by the
// caller (never regrown: captured graphs hold it).
template <typename TV, typename TW>
inline void dot_l(LP<const TV> V, LP<const TW> w, int64_t n, LP<double> out, double *part, hipStream_t s, int K) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_multidot_part<TV, TW>), dim3(nb, K), dim3(kRedBlock), 0, s, V, 0, 1, w, n,
                     LP<double>(part, nb));
  hipLaunchKernelGGL(k_multidot_final, dim3(1, K), dim3(kWave), 0, s, LP<const double>(part, nb), nb, 1, out);
  FSI_CHECK_LAUNCH();
}

// w -= sum_{i<k} h[i] V_i (h on the device), all FP64
__global__ void k_multiaxpy_sub(double *w, const double *V, int64_t ldv, int k, const double *h,
                                int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = w[e];
    for (int i = 0; i < k; ++i) s -= h[i] * V[(int64_t)i * ldv + e];
    w[e] = s;
  }
}

// x += sum_{i<k} y[i] Z_i (y on the device)
__global__ void k_multiaxpy_add(double *x, const double *Z, int64_t ldz, int k, const double *y,
                                int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = x[e];
    for (int i = 0; i < k; ++i) s += y[i] * Z[(int64_t)i * ldz + e];
    x[e] = s;
  }
}

}  // namespace
}  // namespace fsi
