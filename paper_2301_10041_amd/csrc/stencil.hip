// Matrix-free products with A_f on the structured P2 lattice (multigrid smoothing and
// residuals).  Every interior row of A_f = (rho/dt) M_f + K_f is one of four stencils,
// fixed by the parities of the node's lattice coordinates (vertex, horizontal edge,
// vertical edge, diagonal edge); rows of boundary nodes are the identity and columns of
// boundary nodes are zero (the Dirichlet condition imposed by value).  The coefficients
// come from the same element matrices as the assembled A_f (host tables per level), so the
// stencil product equals the CSR product up to the order of the sums.
//
// Bytes per node in the Chebyshev step: x, b, d read, d and y written (5 two-component
// vectors); no matrix and no indices.
#include "ctx.h"
#include "kernels.h"
#include "stencil.h"

namespace fsi {

template <typename T>
struct StencilArgs {
  int n;
  const StencilTable<T> *tab;   // device
  const T *x, *b;
  T *d, *y;
  int L2;                      // nodes per component (2n+1)^2
  T c1, c2;
  // SP_A11 only: fluid rows on [u_x | u_y | p] (x and y hold all three; see
  // stencil_fluid_rows), optional C_f^T x_lam on the velocity rows
  const DivTable<T> *dv;
  const int *cft_rp, *cft_col;
  const T *cft_val, *xlx, *xly;
};

// Tiled kernel.  A block owns kTileR lattice rows x kTileC nodes.  Phase 1 stages x with a
// halo of two nodes into LDS (stride-1, coalesced), storing 0 for boundary nodes and for
// nodes outside the lattice, so that interior rows need no column test.  Phase 2: wave w
// computes row w of the tile, first the even-I nodes then the odd-I nodes, so the node
// class (and the coefficient addresses) are uniform over the wave.  Phase 3 reads the
// products back in row-major order and does the mode's epilogue with coalesced global
// accesses.  Boundary rows are the identity.
constexpr int kTW = kTileC + 4;                 // tile width with halo
constexpr int kTH = kTileR + 4;

template <typename T, int CLS>
__device__ __forceinline__ void tile_row_products(const StencilTable<T> &tb, const T *X0, const T *X1,
                                                  int base, T &s0, T &s1) {
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int k = 0; k < kStencilCount[CLS]; ++k) {
    const int o = base + tb.lds[CLS][k];
    const T y0 = X0[o], y1 = X1[o];
    s0 += tb.coef[CLS][k][0] * y0 + tb.coef[CLS][k][1] * y1;
    s1 += tb.coef[CLS][k][2] * y0 + tb.coef[CLS][k][3] * y1;
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b to XCD b % 8); each XCD
// gets a contiguous band of tiles in row-major order, so the halo rows a tile shares with
// the tile below are still in that XCD's L2.
constexpr int kXcd = 8;

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_stencil(StencilArgs<T> a, int tiles_x, int tiles, int band) {
  __shared__ T X[2][kTH * kTW];
  __shared__ T S[2][kTileR * kTileC];
  const int t = (blockIdx.x % kXcd) * band + blockIdx.x / kXcd;
  if (t >= tiles) return;
  const int n2 = 2 * a.n, L = n2 + 1;
  const int I0 = (t % tiles_x) * kTileC, J0 = (t / tiles_x) * kTileR;
  const int tid = threadIdx.x;
  const StencilTable<T> &tb = *a.tab;
  // phase 1: x tile with halo
  for (int e = tid; e < kTH * kTW; e += 256) {
    const int tr = e / kTW, tc = e % kTW;
    const int I = I0 - 2 + tc, J = J0 - 2 + tr;
    T v0 = 0, v1 = 0;
    if (I > 0 && J > 0 && I < n2 && J < n2) {
      const int r = J * L + I;
      v0 = a.x[r];
      v1 = a.x[a.L2 + r];
    }
    X[0][e] = v0;
    X[1][e] = v1;
  }
  __syncthreads();
  // phase 2: products of the interior rows, one tile row per wave
  {
    const int w = tid / kWave, lane = tid % kWave;
    const int J = J0 + w;
    if (J > 0 && J < n2) {
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const int i = 2 * lane + par;
        const int I = I0 + i;
        T s0 = 0, s1 = 0;
        const int base = (w + 2) * kTW + (i + 2);
        if (I > 0 && I < n2) {
          if (J & 1) {
            if (par) tile_row_products<T, 3>(tb, X[0], X[1], base, s0, s1);
            else tile_row_products<T, 2>(tb, X[0], X[1], base, s0, s1);
          } else {
            if (par) tile_row_products<T, 1>(tb, X[0], X[1], base, s0, s1);
            else tile_row_products<T, 0>(tb, X[0], X[1], base, s0, s1);
          }
        }
        S[0][w * kTileC + i] = s0;
        S[1][w * kTileC + i] = s1;
      }
    }
  }
  __syncthreads();
  // phase 3: epilogue, row-major and coalesced
  for (int e = tid; e < kTileR * kTileC; e += 256) {
    const int j = e / kTileC, i = e % kTileC;
    const int I = I0 + i, J = J0 + j;
    if (I > n2 || J > n2) continue;
    const int r = J * L + I;
    const bool bnd = I == 0 || J == 0 || I == n2 || J == n2;
    const T x0 = a.x[r], x1 = a.x[a.L2 + r];
    const T s0 = bnd ? x0 : S[0][e], s1 = bnd ? x1 : S[1][e];
    if constexpr (MODE == SP_APPLY) {
      a.y[r] = s0;
      a.y[a.L2 + r] = s1;
    } else if constexpr (MODE == SP_A11) {
      T t0 = s0, t1 = s1;
      if (!bnd) {   // - B^T x_p; column 0 (pinned pressure) is zero
        const DivTable<T> &dv = *a.dv;
        const T *xp = a.x + 2 * (int64_t)a.L2;
        const int cls = (I & 1) | ((J & 1) << 1);
        const int pi = I >> 1, pj = J >> 1, L1 = a.n + 1;
        for (int k = 0; k < dv.bt_count[cls]; ++k) {
          const int q = (pj + dv.bt_off[cls][k][1]) * L1 + pi + dv.bt_off[cls][k][0];
          const T pv = q == 0 ? T(0) : xp[q];
          t0 -= dv.bt_coef[cls][k][0] * pv;
          t1 -= dv.bt_coef[cls][k][1] * pv;
        }
      }
      if (a.cft_rp) {
        for (int k = a.cft_rp[r]; k < a.cft_rp[r + 1]; ++k) {
          const T cv = a.cft_val[k];
          const int j = a.cft_col[k];
          t0 += cv * a.xlx[j];
          t1 += cv * a.xly[j];
        }
      }
      a.y[r] = t0;
      a.y[a.L2 + r] = t1;
    } else if constexpr (MODE == SP_RESID) {
      a.y[r] = a.b[r] - s0;
      a.y[a.L2 + r] = a.b[a.L2 + r] - s1;
    } else {
      const T r0 = a.b[r] - s0, r1 = a.b[a.L2 + r] - s1;
      T z0 = r0, z1 = r1;
      if (!bnd) {
        const int cls = (I & 1) | ((J & 1) << 1);
        z0 = tb.dinv[cls][0] * r0 + tb.dinv[cls][1] * r1;
        z1 = tb.dinv[cls][2] * r0 + tb.dinv[cls][3] * r1;
      }
      const T d0 = a.c1 * a.d[r] + a.c2 * z0, d1 = a.c1 * a.d[a.L2 + r] + a.c2 * z1;
      a.d[r] = d0;
      a.d[a.L2 + r] = d1;
      a.y[r] = x0 + d0;
      a.y[a.L2 + r] = x1 + d1;
    }
  }
  if constexpr (MODE == SP_A11) {
    // phase 4: pressure rows of the P1 nodes at even lattice positions of the tile
    // (2 rows x 64 nodes), -B x_u from the staged x tile (Dirichlet values read as zero)
    if (tid < 2 * kWave) {
      const int pr = tid / kWave, pc = tid % kWave;
      const int pi = (I0 >> 1) + pc, pj = (J0 >> 1) + pr;
      if (pi <= a.n && pj <= a.n) {
        const DivTable<T> &dv = *a.dv;
        const int base = (2 * pr + 2) * kTW + (2 * pc + 2);
        T sp = 0;
        for (int k = 0; k < dv.b_count; ++k) {
          const int o = base + dv.b_lds[k];
          sp += dv.b_coef[k][0] * X[0][o] + dv.b_coef[k][1] * X[1][o];
        }
        const int64_t q = (int64_t)pj * (a.n + 1) + pi;
        const int64_t o2 = 2 * (int64_t)a.L2;
        a.y[o2 + q] = q == 0 ? a.x[o2] : -sp;
      }
    }
  }
}

template <typename T, int MODE>
static void launch_tiles(int n, const StencilArgs<T> &a, hipStream_t s) {
  const int L = 2 * n + 1;
  const int tx = (L + kTileC - 1) / kTileC, ty = (L + kTileR - 1) / kTileR;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  hipLaunchKernelGGL((k_stencil<T, MODE>), dim3((unsigned)(band * kXcd)), dim3(256), 0, s, a, tx, tiles, band);
  FSI_CHECK_LAUNCH();
}

template <typename T, int MODE>
void stencil_launch(int n, const StencilTable<T> *tab, const T *x, const T *b, T *d, T *y, T c1, T c2,
                    hipStream_t s) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  static_assert(kTileR * kWave == 256 && 2 * kWave == kTileC, "one tile row per wave, two nodes per lane");
  StencilArgs<T> a{n, tab, x, b, d, y, (2 * n + 1) * (2 * n + 1), c1, c2, nullptr, nullptr, nullptr,
                   nullptr, nullptr, nullptr};
  launch_tiles<T, MODE>(n, a, s);
}

template <typename T>
void stencil_fluid_rows(int n, const StencilTable<T> *tab, const DivTable<T> *dv, const T *x, T *y,
                        const int *cft_rp, const int *cft_col, const T *cft_val, const T *xl, int64_t Ns,
                        hipStream_t s) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  static_assert(kTileC % 2 == 0 && kTileR % 2 == 0 && kTileC / 2 == kWave && kTileR / 2 * kWave <= 256,
                "a tile holds 2 x 64 P1 nodes, one per thread of the first two waves");
  const int L = 2 * n + 1, L2 = L * L;
  StencilArgs<T> a{n, tab, x, nullptr, nullptr, y, L2, T(0), T(0), dv, cft_rp, cft_col, cft_val, xl,
                   xl ? xl + Ns : nullptr};
  launch_tiles<T, SP_A11>(n, a, s);
}
template void stencil_fluid_rows<double>(int, const StencilTable<double> *, const DivTable<double> *,
                                         const double *, double *, const int *, const int *, const double *,
                                         const double *, int64_t, hipStream_t);
template void stencil_fluid_rows<float>(int, const StencilTable<float> *, const DivTable<float> *, const float *,
                                        float *, const int *, const int *, const float *, const float *, int64_t,
                                        hipStream_t);

template void stencil_launch<double, SP_APPLY>(int, const StencilTable<double> *, const double *, const double *,
                                               double *, double *, double, double, hipStream_t);
template void stencil_launch<double, SP_RESID>(int, const StencilTable<double> *, const double *, const double *,
                                               double *, double *, double, double, hipStream_t);
template void stencil_launch<double, SP_CHEB>(int, const StencilTable<double> *, const double *, const double *,
                                              double *, double *, double, double, hipStream_t);
template void stencil_launch<float, SP_APPLY>(int, const StencilTable<float> *, const float *, const float *,
                                              float *, float *, float, float, hipStream_t);
template void stencil_launch<float, SP_RESID>(int, const StencilTable<float> *, const float *, const float *,
                                              float *, float *, float, float, hipStream_t);
template void stencil_launch<float, SP_CHEB>(int, const StencilTable<float> *, const float *, const float *,
                                             float *, float *, float, float, hipStream_t);

}  // namespace fsi
