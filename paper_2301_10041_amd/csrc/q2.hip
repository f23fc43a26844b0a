// Class stencils of the paper's element pair (Q2 velocity, discontinuous P1 pressure) and the
// smoothing kernel of its velocity V-cycle that uses them (the Q2 A_f rows by class).
#include <algorithm>
#include <cstring>

#include "ctx.h"
#include "kernels.h"
#include "q2.h"

namespace fsi {

// Class stencils of the Q2 A_f: the row of an interior node of each class summed over its cells
// as k_asm_q2q2 sums them (node (2 + a, 2 + b) of class a + 2 b has every cell inside for n >= 2).
void q2_tables(int n, double nu, double rdt, Q2Table<double> &t64, Q2Table<float> &t32) {
  FSI_REQUIRE(n >= 2, FSI_E_ARG, "Q2 class stencils need n >= 2");
  std::vector<double> E;
  q2_element_table(n, nu, E);
  std::memset(&t64, 0, sizeof(t64));
  std::memset(&t32, 0, sizeof(t32));
  for (int cls = 0; cls < 4; ++cls) {
    const int I = 2 + (cls & 1), J = 2 + (cls >> 1);
    const int i0 = std::max(0, (I - 1) >> 1), i1 = std::min(n - 1, I >> 1);
    const int j0 = std::max(0, (J - 1) >> 1), j1 = std::min(n - 1, J >> 1);
    int cnt = 0;
    for (int J2 = 2 * j0; J2 <= 2 * j1 + 2; ++J2)
      for (int I2 = 2 * i0; I2 <= 2 * i1 + 2; ++I2) {
        double m = 0.0, kk[4] = {0.0, 0.0, 0.0, 0.0};
        for (int cj = j0; cj <= j1; ++cj) {
          const int b = J - 2 * cj, b2 = J2 - 2 * cj;
          if (b2 < 0 || b2 > 2) continue;
          for (int ci = i0; ci <= i1; ++ci) {
            const int a = I - 2 * ci, a2 = I2 - 2 * ci;
            if (a2 < 0 || a2 > 2) continue;
            const int li = a + 3 * b, lj = a2 + 3 * b2;
            m += E[QE_M + 9 * li + lj];
            for (int q = 0; q < 4; ++q) kk[q] += E[QE_K + (q * 9 + li) * 9 + lj];
          }
        }
        FSI_REQUIRE(cnt < kQ2Max, FSI_E_ARG, "Q2 stencil too wide");
        const double v[4] = {rdt * m + kk[0], kk[1], kk[2], rdt * m + kk[3]};
        t64.off[cls][cnt][0] = t32.off[cls][cnt][0] = I2 - I;
        t64.off[cls][cnt][1] = t32.off[cls][cnt][1] = J2 - J;
        const int dk = (I2 - I + 2) + 5 * (J2 - J + 2);
        for (int q = 0; q < 4; ++q) {
          t64.coef[cls][cnt][q] = t64.dense[cls][dk][q] = v[q];
          t32.coef[cls][cnt][q] = t32.dense[cls][dk][q] = (float)v[q];
        }
        if (I2 == I && J2 == J) {
          const double det = v[0] * v[3] - v[1] * v[2];
          const double di[4] = {v[3] / det, -v[1] / det, -v[2] / det, v[0] / det};
          for (int q = 0; q < 4; ++q) {
            t64.dinv[cls][q] = di[q];
            t32.dinv[cls][q] = (float)di[q];
          }
        }
        ++cnt;
      }
    t64.count[cls] = t32.count[cls] = cnt;
  }
}

// A tile of kQ2TW x kQ2TH lattice nodes per workgroup, one thread per node: x of the tile and a
// halo of two nodes staged in LDS (two components; Dirichlet and outside nodes stored as zero,
// which leaves them out of every row), the class's 2 x 2 blocks on the full 5 x 5 window with
// compile-time LDS offsets (the entries a class lacks are zero).  Boundary rows: the identity.
constexpr int kQ2TW = 64, kQ2TH = 4, kQ2SW = kQ2TW + 4, kQ2SH = kQ2TH + 4;
template <typename T, bool RESID>
__global__ void __launch_bounds__(kQ2TW * kQ2TH) k_q2_stencil(int n, const Q2Table<T> *__restrict__ tab,
                                                             const T *__restrict__ x, const T *__restrict__ b,
                                                             T *__restrict__ d, T *__restrict__ y, T c1, T c2) {
  __shared__ T cs[4][25][4];
  __shared__ T dv[4][4];
  __shared__ T xs[2][kQ2SH * kQ2SW];
  const int tid = threadIdx.x;
  for (int k = tid; k < 4 * 25 * 4; k += kQ2TW * kQ2TH) (&cs[0][0][0])[k] = (&tab->dense[0][0][0])[k];
  if (tid < 16) (&dv[0][0])[tid] = (&tab->dinv[0][0])[tid];
  const int64_t L = 2 * n + 1, N = L * L;
  const int I0 = blockIdx.x * kQ2TW, J0 = blockIdx.y * kQ2TH;
  for (int k = tid; k < kQ2SH * kQ2SW; k += kQ2TW * kQ2TH) {
    const int I = I0 - 2 + k % kQ2SW, J = J0 - 2 + k / kQ2SW;
    const bool in = I > 0 && J > 0 && I < 2 * n && J < 2 * n;
    const int64_t j = (int64_t)J * L + I;
    xs[0][k] = in ? x[j] : (T)0;
    xs[1][k] = in ? x[N + j] : (T)0;
  }
  __syncthreads();
  const int tx = tid % kQ2TW, ty = tid / kQ2TW;
  const int I = I0 + tx, J = J0 + ty;
  if (I >= L || J >= L) return;
  const int64_t r = (int64_t)J * L + I;
  T r0, r1, z0, z1;
  if (I == 0 || J == 0 || I == 2 * n || J == 2 * n) {
    r0 = b[r] - x[r];
    r1 = b[N + r] - x[N + r];
    z0 = r0;
    z1 = r1;
  } else {
    const int cls = (I & 1) + 2 * (J & 1);
    const T(*c)[4] = cs[cls];
    const T *x0p = &xs[0][ty * kQ2SW + tx], *x1p = &xs[1][ty * kQ2SW + tx];
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int dJ = 0; dJ < 5; ++dJ)
#pragma unroll
      for (int dI = 0; dI < 5; ++dI) {
        const int k = dI + 5 * dJ, o = dJ * kQ2SW + dI;
        const T x0 = x0p[o], x1 = x1p[o];
        s0 += c[k][0] * x0 + c[k][1] * x1;
        s1 += c[k][2] * x0 + c[k][3] * x1;
      }
    r0 = b[r] - s0;
    r1 = b[N + r] - s1;
    z0 = dv[cls][0] * r0 + dv[cls][1] * r1;
    z1 = dv[cls][2] * r0 + dv[cls][3] * r1;
  }
  if constexpr (RESID) {
    y[r] = r0;
    y[N + r] = r1;
  } else {
    const T d0 = c1 * d[r] + c2 * z0, d1 = c1 * d[N + r] + c2 * z1;
    d[r] = d0;
    d[N + r] = d1;
    y[r] = x[r] + d0;
    y[N + r] = x[N + r] + d1;
  }
}

template <typename T>
void q2_stencil(int n, const Q2Table<T> *tab, const T *x, const T *b, T *d, T *y, T c1, T c2, bool resid,
                hipStream_t s) {
  const int L = 2 * n + 1;
  const dim3 grid((unsigned)((L + kQ2TW - 1) / kQ2TW), (unsigned)((L + kQ2TH - 1) / kQ2TH));
  if (resid)
    hipLaunchKernelGGL((k_q2_stencil<T, true>), grid, dim3(kQ2TW * kQ2TH), 0, s, n, tab, x, b, d, y, c1, c2);
  else
    hipLaunchKernelGGL((k_q2_stencil<T, false>), grid, dim3(kQ2TW * kQ2TH), 0, s, n, tab, x, b, d, y, c1, c2);
  FSI_CHECK_LAUNCH();
}
template void q2_stencil<double>(int, const Q2Table<double> *, const double *, const double *, double *, double *,
                                 double, double, bool, hipStream_t);
template void q2_stencil<float>(int, const Q2Table<float> *, const float *, const float *, float *, float *, float,
                                float, bool, hipStream_t);

}  // namespace fsi
