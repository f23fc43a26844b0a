// The coarse end of the pressure (P1) V-cycle in one launch per system (Sec. 4 multigrid,
// the Cahouet-Chabard Schur preconditioner).  On levels of at most 64 x 64 cells the
// per-level launches (smoothing, residual, restriction, prolongation) cost the latency of a
// kernel each for a few thousand nodes.  One 1024-thread block keeps every remaining level in
// LDS and runs the steps of those launches with block barriers between passes: the Chebyshev
// steps of k_p1_multi (same coefficients, same order of the stencil sums, the pinned row and
// column), the residual of k_p1, the restriction of k_p1_restrict, the dense coarsest solve
// of k_dense_mv and the linear prolongation of k_p1_prolong_add.  Node r of a level belongs
// to thread r mod 1024 in every pass, so its search direction stays in that thread's
// registers.
#include "ctx.h"
#include "kernels.h"
#include "lattice.h"

namespace fsi {

namespace {

constexpr int kTailThreads = 1024;

// (A x)_r on a P1 level of n cells (row-major x, side L = n + 1), as k_p1 sums it
template <typename T>
__device__ __forceinline__ T p1_apply(const T *tb, int pin, const T *x, int n, int r) {
  const int L = n + 1, i = r % L, j = r / L;
  const T xc = x[r];
  if (pin && r == 0) return xc;   // identity row of the pinned node
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  const T *c = tb + kP1Nbr * (3 * cj + ci);
  // column 0 is zero when pinned: node (0, 0) is read as 0
  auto ld = [&](int q) -> T { return (pin && q == 0) ? T(0) : x[q]; };
  T s = c[0] * xc;
  if (i > 0) s += c[1] * ld(r - 1);
  if (i < n) s += c[2] * x[r + 1];
  if (j > 0) s += c[3] * ld(r - L);
  if (j < n) s += c[4] * x[r + L];
  if (i > 0 && j > 0) s += c[5] * ld(r - L - 1);
  if (i < n && j < n) s += c[6] * x[r + L + 1];
  return s;
}

template <typename T>
__device__ __forceinline__ T p1_dinv(const T *tb, int n, int r) {
  const int L = n + 1, i = r % L, j = r / L;
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  return tb[9 * kP1Nbr + 3 * cj + ci];
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_p1_tail(PTailArgs<T> a) {
  extern __shared__ unsigned char ptail_smem[];
  T *sm = reinterpret_cast<T *>(ptail_smem);
  const int tid = threadIdx.x;
  const T *bg = a.b + (int64_t)blockIdx.y * a.lb;
  T *xg = a.x + (int64_t)blockIdx.y * a.lb;
  {   // the first level's right-hand side, the tables, the dense inverse (when in LDS)
    const int L0 = a.lv[0].n + 1, N0 = L0 * L0;
    for (int r = tid; r < N0; r += kTailThreads) sm[a.lv[0].off + r] = bg[r];
    for (int l = 0; l < a.nlev; ++l)
      for (int i = tid; i < kPTailTab; i += kTailThreads) {
        const P1Table<T> &tb = *a.lv[l].tab;
        sm[a.offt + l * kPTailTab + i] = i < 9 * kP1Nbr ? tb.coef[i / kP1Nbr][i % kP1Nbr] : tb.dinv[i - 9 * kP1Nbr];
      }
    if (a.offm >= 0)
      for (int i = tid; i < a.m * a.m; i += kTailThreads) sm[a.offm + i] = a.cinv[i];
  }
  __syncthreads();
  T *x2 = sm + a.offx2;
  T dreg[kPTailPer];
  // S Chebyshev steps on level l from zero (ZERO) or from its x; the result ends in x
  auto smooth = [&](int l, bool zero) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, N = (n + 1) * (n + 1);
    const T *tb = sm + a.offt + l * kPTailTab;
    const int pin = lv.tab->pin;
    T *b = sm + lv.off, *x = b + N;
    int k0 = 0;
    if (zero) {   // x = d = c2[0] D^{-1} b
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) {
        const int r = tid + kTailThreads * q;
        if (r < N) {
          const T z = lv.c2[0] * (p1_dinv(tb, n, r) * b[r]);
          dreg[q] = z;
          x[r] = z;
        }
      }
      k0 = 1;
      __syncthreads();
    } else {
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) dreg[q] = T(0);
    }
    T *src = x, *dst = x2;
    for (int k = k0; k < a.degree; ++k) {
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) {
        const int r = tid + kTailThreads * q;
        if (r < N) {
          const T sum = p1_apply(tb, pin, src, n, r);
          const T z = p1_dinv(tb, n, r) * (b[r] - sum);
          const T dn = lv.c1[k] * dreg[q] + lv.c2[k] * z;
          dreg[q] = dn;
          dst[r] = src[r] + dn;
        }
      }
      __syncthreads();
      T *t = src;
      src = dst;
      dst = t;
    }
    if (src != x) {   // an odd number of steps from x left the result in the second buffer
      for (int r = tid; r < N; r += kTailThreads) x[r] = src[r];
      __syncthreads();
    }
  };
  // descent: pre-smoothing, residual (into the second buffer), restriction
  for (int l = 0; l < a.nlev; ++l) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, L = n + 1, N = L * L;
    const T *tb = sm + a.offt + l * kPTailTab;
    T *b = sm + lv.off, *x = b + N;
    smooth(l, true);
    const int pin = lv.tab->pin;
    for (int r = tid; r < N; r += kTailThreads) x2[r] = b[r] - p1_apply(tb, pin, x, n, r);
    __syncthreads();
    const int nc = n / 2, Lc = nc + 1;
    const bool coarsest = l + 1 == a.nlev;
    T *bc = coarsest ? sm + a.offc : sm + a.lv[l + 1].off;
    for (int q = tid; q < Lc * Lc; q += kTailThreads) {
      if (q == 0) {
        bc[0] = T(0);
        continue;
      }
      const int fi = 2 * (q % Lc), fj = 2 * (q / Lc);
      auto fv = [&](int u, int v) -> T {
        if (u < 0 || v < 0 || u > n || v > n) return T(0);
        const int f = v * L + u;
        return f == 0 ? T(0) : x2[f];
      };
      const T edges = fv(fi - 1, fj) + fv(fi + 1, fj) + fv(fi, fj - 1) + fv(fi, fj + 1) + fv(fi + 1, fj + 1) +
                      fv(fi - 1, fj - 1);
      bc[q] = fv(fi, fj) + T(0.5) * edges;
    }
    __syncthreads();
  }
  {   // coarsest level: x = C^{-1} b, one wave per row, sums in double (as k_dense_mv)
    const T *b = sm + a.offc;
    T *x = sm + a.offc + a.m;
    const T *cm = a.offm >= 0 ? sm + a.offm : a.cinv;
    const int w = tid / kWave, lane = tid % kWave;
    for (int r = w; r < a.m; r += kTailThreads / kWave) {
      double s = 0.0;
      for (int k = lane; k < a.m; k += kWave) s += (double)cm[(int64_t)r * a.m + k] * (double)b[k];
      s = wave_sum(s);
      if (lane == 0) x[r] = (T)s;
    }
  }
  __syncthreads();
  // ascent: linear prolongation of the coarse correction (the pinned node excluded), post-smoothing
  for (int l = a.nlev - 1; l >= 0; --l) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, L = n + 1, N = L * L, Lc = n / 2 + 1;
    T *x = sm + lv.off + N;
    const T *xc = l + 1 == a.nlev ? sm + a.offc + a.m : sm + a.lv[l + 1].off + Lc * Lc;
    for (int r = tid; r < N; r += kTailThreads) {
      if (r == 0) continue;
      const int i = r % L, j = r / L, ci = i >> 1, cj = j >> 1;
      auto cv = [&](int u, int v) -> T {
        const int k = v * Lc + u;
        return k == 0 ? T(0) : xc[k];
      };
      T s;
      if (!(i & 1) && !(j & 1)) s = cv(ci, cj);
      else if (!(j & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj);
      else if (!(i & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci, cj + 1);
      else s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj + 1);
      x[r] += s;
    }
    __syncthreads();
    smooth(l, false);
  }
  {
    const int N0 = (a.lv[0].n + 1) * (a.lv[0].n + 1);
    const T *x = sm + a.lv[0].off + N0;
    for (int r = tid; r < N0; r += kTailThreads) xg[r] = x[r];
  }
}

}  // namespace

int tail_lds_limit() {
  static int limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    v = v < 65536 ? v : v > 163840 ? 163840 : v;
    // dynamic LDS above 64 KiB is granted per kernel
    if (v > 65536 && (hipFuncSetAttribute((const void *)k_p1_tail<double>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess ||
                      hipFuncSetAttribute((const void *)k_p1_tail<float>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess)) {
      (void)hipGetLastError();
      v = 65536;
    }
    return v;
  }();
  return limit;
}

template <typename T>
void p1_tail(const PTailArgs<T> &a, hipStream_t s, int K) {
  FSI_REQUIRE(a.nlev >= 1 && a.nlev <= kPTailMax && a.degree >= 1 && a.degree <= kPTailDeg, FSI_E_ARG,
              "pressure tail shape out of range");
  FSI_REQUIRE(a.lv[0].n <= kPTailMaxN && (a.lv[0].n + 1) * (a.lv[0].n + 1) <= kPTailPer * kTailThreads, FSI_E_ARG,
              "pressure tail level too fine");
  for (int l = 0; l + 1 < a.nlev; ++l)
    FSI_REQUIRE(a.lv[l + 1].n * 2 == a.lv[l].n, FSI_E_ARG, "pressure tail levels not nested");
  FSI_REQUIRE(a.m == (a.lv[a.nlev - 1].n / 2 + 1) * (a.lv[a.nlev - 1].n / 2 + 1) && a.m <= kPTailDenseMax, FSI_E_ARG,
              "pressure tail coarsest level out of range");
  FSI_REQUIRE(K >= 1 && K <= 65535 && (K == 1 || a.lb > 0), FSI_E_ARG, "lane count out of range");
  const int bytes = a.lds * (int)sizeof(T);
  FSI_REQUIRE(bytes <= tail_lds_limit(), FSI_E_ARG, "pressure tail exceeds the LDS of a block");
  hipLaunchKernelGGL(k_p1_tail<T>, dim3(1, (unsigned)K), dim3(kTailThreads), bytes, s, a);
  FSI_CHECK_LAUNCH();
}
template void p1_tail<double>(const PTailArgs<double> &, hipStream_t, int);
template void p1_tail<float>(const PTailArgs<float> &, hipStream_t, int);

}  // namespace fsi
