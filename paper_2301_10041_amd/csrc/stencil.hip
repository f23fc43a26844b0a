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
#include <initializer_list>
#include <type_traits>
#include <utility>

#include "ctx.h"
#include "kernels.h"
#include "lattice.h"
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
  // SP_A11 inside MINRES (ms_s set): with device scalars s = *ms_s, c = *ms_c, write
  // v = s x and y = s (A11 x) + c r1 over r1 (ms_r1y; r1 read only where c != 0), and the
  // block's part of v . y to ms_part[tile]
  const double *ms_s, *ms_c;
  T *ms_v, *ms_r1y;
  double *ms_part;
  // lane strides (blockIdx.y = lane): vectors, MINRES scalars, per-tile parts.  The C_f^T
  // term (cft_*, xlx, xly) is one system's and is not shifted.
  int64_t lv, ls, lp;
  // in MINRES: ms_v is the base of the Lanczos block; v goes to slot *ms_slot (a device
  // scalar of the lane's state, clamped to [0, ms_nslot - 1]) at stride ms_vs
  const double *ms_slot;
  int64_t ms_vs;
  int ms_nslot;
};

// Views of lane blockIdx.y (null pointers stay null).
template <typename P>
__device__ __forceinline__ void lane_shift(P *&p, int64_t stride) {
  if (p) p += (int64_t)blockIdx.y * stride;
}
template <typename T>
__device__ __forceinline__ StencilArgs<T> lane_args(const StencilArgs<T> &a0) {
  StencilArgs<T> a = a0;
  lane_shift(a.x, a.lv);
  lane_shift(a.b, a.lv);
  lane_shift(a.d, a.lv);
  lane_shift(a.y, a.lv);
  lane_shift(a.ms_v, a.lv);
  lane_shift(a.ms_r1y, a.lv);
  lane_shift(a.ms_s, a.ls);
  lane_shift(a.ms_c, a.ls);
  lane_shift(a.ms_part, a.lp);
  lane_shift(a.ms_slot, a.ls);
  if (a.ms_slot) {
    int sl = (int)*a.ms_slot;
    sl = sl < 0 ? 0 : sl >= a.ms_nslot ? a.ms_nslot - 1 : sl;
    a.ms_v += (int64_t)sl * a.ms_vs;
  }
  return a;
}

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
  constexpr StencilOffsets so = stencil_offsets();
  constexpr CrossZero cz = cross_zero();
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int k = 0; k < kStencilCount[CLS]; ++k) {
    const int o = base + so.d[CLS][k][1] * kTW + so.d[CLS][k][0];
    const T y0 = X0[o], y1 = X1[o];
    if (cz.z[CLS][k]) {   // xy = yx = 0 (fma with a zero coefficient adds nothing)
      s0 = fma(tb.coef[CLS][k][0], y0, s0);
      s1 = fma(tb.coef[CLS][k][3], y1, s1);
    } else {
      s0 = fma(tb.coef[CLS][k][1], y1, fma(tb.coef[CLS][k][0], y0, s0));
      s1 = fma(tb.coef[CLS][k][3], y1, fma(tb.coef[CLS][k][2], y0, s1));
    }
  }
}

// B^T x_p of a class-CLS node from the staged pressure tile (row width kPW), base = the
// tile position of P1 node (I >> 1, J >> 1)
constexpr int kPW = kTileC / 2 + 2, kPH = kTileR / 2 + 2;   // P1 tile with a halo of one
template <typename T, int CLS>
__device__ __forceinline__ void tile_bt_products(const DivTable<T> &dv, const T *XP, int base, T &s0, T &s1) {
  constexpr DivOffsets so = div_offsets();
#pragma unroll
  for (int k = 0; k < kBtCount[CLS]; ++k) {
    const T pv = XP[base + so.bt[CLS][k][1] * kPW + so.bt[CLS][k][0]];
    s0 = fma(-dv.bt_coef[CLS][k][0], pv, s0);
    s1 = fma(-dv.bt_coef[CLS][k][1], pv, s1);
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b to XCD b % 8); each XCD
// gets a contiguous band of tiles in row-major order, so the halo rows a tile shares with
// the tile below are still in that XCD's L2.
constexpr int kXcd = 8;

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_stencil(StencilArgs<T> a0, int tiles_x, int tiles, int band) {
  __shared__ T X[2][kTH * kTW];
  __shared__ T S[2][kTileR * kTileC];
  __shared__ T XP[MODE == SP_A11 ? kPH * kPW : 1];   // SP_A11: x_p tile (column 0 read as 0)
  const int t = (blockIdx.x % kXcd) * band + blockIdx.x / kXcd;
  if (t >= tiles) return;
  const StencilArgs<T> a = lane_args(a0);
  const int n2 = 2 * a.n, L = n2 + 1;
  const int I0 = (t % tiles_x) * kTileC, J0 = (t / tiles_x) * kTileR;
  const int tid = threadIdx.x;
  const StencilTable<T> &tb = *a.tab;
  double ms_acc = 0.0;   // SP_A11 in MINRES: this thread's part of v . y
  // epilogue operands of this thread's nodes (row-major, coalesced), loaded first; x only at
  // Dirichlet nodes (the staged tile holds 0 there), the interior x comes from the tile
  constexpr int EIT = kTileR * kTileC / 256;
  T ex[EIT][2], eb[EIT][2], ed[EIT][2];
#pragma unroll
  for (int q = 0; q < EIT; ++q) {
    const int e = tid + 256 * q, I = I0 + e % kTileC, J = J0 + e / kTileC;
    ex[q][0] = ex[q][1] = eb[q][0] = eb[q][1] = ed[q][0] = ed[q][1] = 0;
    if (I <= n2 && J <= n2) {
      const int r = J * L + I;
      if (I == 0 || J == 0 || I == n2 || J == n2) {
        ex[q][0] = a.x[r];
        ex[q][1] = a.x[a.L2 + r];
      }
      if constexpr (MODE == SP_RESID || MODE == SP_CHEB) {
        eb[q][0] = a.b[r];
        eb[q][1] = a.b[a.L2 + r];
      }
      if constexpr (MODE == SP_CHEB) {
        ed[q][0] = a.d[r];
        ed[q][1] = a.d[a.L2 + r];
      }
      if constexpr (MODE == SP_A11) {   // in MINRES: r1 (ed holds it)
        if (a.ms_s) {
          ed[q][0] = a.ms_r1y[r];
          ed[q][1] = a.ms_r1y[a.L2 + r];
        }
      }
    }
  }
  // SP_A11: the pressure tile (P1 rows J0/2 - 1 .. J0/2 + 2, columns I0/2 - 1 .. I0/2 + 64)
  // and, for the pressure rows of the tile (threads 0..127), x_p and r1 at the own node
  T pp_x = 0, pp_r1 = 0;
  if constexpr (MODE == SP_A11) {
    const int64_t o2 = 2 * (int64_t)a.L2;
    for (int e = tid; e < kPH * kPW; e += 256) {
      const int pi = (I0 >> 1) - 1 + e % kPW, pj = (J0 >> 1) - 1 + e / kPW;
      T pv = 0;
      if (pi >= 0 && pj >= 0 && pi <= a.n && pj <= a.n) {
        const int64_t q = (int64_t)pj * (a.n + 1) + pi;
        if (q != 0) pv = a.x[o2 + q];
      }
      XP[e] = pv;
    }
    if (tid < 2 * kWave) {
      const int pi = (I0 >> 1) + tid % kWave, pj = (J0 >> 1) + tid / kWave;
      if (pi <= a.n && pj <= a.n) {
        const int64_t q = (int64_t)pj * (a.n + 1) + pi;
        pp_x = a.x[o2 + q];
        if (a.ms_s) pp_r1 = a.ms_r1y[o2 + q];
      }
    }
  }
  // phase 1: x tile with halo (all loads issued before the LDS stores)
  constexpr int NE = kTH * kTW, IT = (NE + 255) / 256;
  T v[IT][2];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + 256 * q, tr = e / kTW, tc = e % kTW;
    const int I = I0 - 2 + tc, J = J0 - 2 + tr;
    v[q][0] = 0;
    v[q][1] = 0;
    if (e < NE && I > 0 && J > 0 && I < n2 && J < n2) {
      const int r = J * L + I;
      v[q][0] = a.x[r];
      v[q][1] = a.x[a.L2 + r];
    }
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + 256 * q;
    if (e < NE) {
      X[0][e] = v[q][0];
      X[1][e] = v[q][1];
    }
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
          // SP_A11: - B^T x_p from the pressure tile; P1 node (I >> 1, J >> 1) sits at
          // tile row (w >> 1) + 1, column lane + 1 (I0 and J0 are even)
          const int pbase = ((w >> 1) + 1) * kPW + lane + 1;
          if (J & 1) {
            if (par) {
              tile_row_products<T, 3>(tb, X[0], X[1], base, s0, s1);
              if constexpr (MODE == SP_A11) tile_bt_products<T, 3>(*a.dv, XP, pbase, s0, s1);
            } else {
              tile_row_products<T, 2>(tb, X[0], X[1], base, s0, s1);
              if constexpr (MODE == SP_A11) tile_bt_products<T, 2>(*a.dv, XP, pbase, s0, s1);
            }
          } else {
            if (par) {
              tile_row_products<T, 1>(tb, X[0], X[1], base, s0, s1);
              if constexpr (MODE == SP_A11) tile_bt_products<T, 1>(*a.dv, XP, pbase, s0, s1);
            } else {
              tile_row_products<T, 0>(tb, X[0], X[1], base, s0, s1);
              if constexpr (MODE == SP_A11) tile_bt_products<T, 0>(*a.dv, XP, pbase, s0, s1);
            }
          }
        }
        S[0][w * kTileC + i] = s0;
        S[1][w * kTileC + i] = s1;
      }
    }
  }
  __syncthreads();
  // phase 3: epilogue, row-major and coalesced
#pragma unroll
  for (int q = 0; q < EIT; ++q) {
    const int e = tid + 256 * q;
    const int j = e / kTileC, i = e % kTileC;
    const int I = I0 + i, J = J0 + j;
    if (I > n2 || J > n2) continue;
    const int r = J * L + I;
    const bool bnd = I == 0 || J == 0 || I == n2 || J == n2;
    const int xo = (j + 2) * kTW + (i + 2);   // the node in the staged tile
    const T x0 = bnd ? ex[q][0] : X[0][xo], x1 = bnd ? ex[q][1] : X[1][xo];
    const T s0 = bnd ? x0 : S[0][e], s1 = bnd ? x1 : S[1][e];
    if constexpr (MODE == SP_APPLY) {
      a.y[r] = s0;
      a.y[a.L2 + r] = s1;
    } else if constexpr (MODE == SP_A11) {
      T t0 = s0, t1 = s1;   // A_f x_u - B^T x_p (identity on Dirichlet rows)
      if (a.cft_rp) {
        for (int k = a.cft_rp[r]; k < a.cft_rp[r + 1]; ++k) {
          const T cv = a.cft_val[k];
          const int j = a.cft_col[k];
          t0 += cv * a.xlx[j];
          t1 += cv * a.xly[j];
        }
      }
      if (a.ms_s) {
        const T sc = (T)*a.ms_s, cc = (T)*a.ms_c;
        T y0 = sc * t0, y1 = sc * t1;
        if (cc != T(0)) {
          y0 += cc * ed[q][0];
          y1 += cc * ed[q][1];
        }
        const T v0 = sc * x0, v1 = sc * x1;
        a.ms_r1y[r] = y0;
        a.ms_r1y[a.L2 + r] = y1;
        a.ms_v[r] = v0;
        a.ms_v[a.L2 + r] = v1;
        ms_acc += (double)v0 * (double)y0 + (double)v1 * (double)y1;
      } else {
        a.y[r] = t0;
        a.y[a.L2 + r] = t1;
      }
    } else if constexpr (MODE == SP_RESID) {
      a.y[r] = eb[q][0] - s0;
      a.y[a.L2 + r] = eb[q][1] - s1;
    } else {
      const T r0 = eb[q][0] - s0, r1 = eb[q][1] - s1;
      T z0 = r0, z1 = r1;
      if (!bnd) {   // class-wise D^{-1}: scalar loads, picked per node
        const int cls = (I & 1) | ((J & 1) << 1);
        T di[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          di[k] = cls == 0 ? tb.dinv[0][k] : cls == 1 ? tb.dinv[1][k] : cls == 2 ? tb.dinv[2][k] : tb.dinv[3][k];
        z0 = di[0] * r0 + di[1] * r1;
        z1 = di[2] * r0 + di[3] * r1;
      }
      const T d0 = a.c1 * ed[q][0] + a.c2 * z0, d1 = a.c1 * ed[q][1] + a.c2 * z1;
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
        constexpr StencilOffsets so = stencil_offsets();   // B rows: the vertex pattern
        const int base = (2 * pr + 2) * kTW + (2 * pc + 2);
        T sp = 0;
#pragma unroll
        for (int k = 0; k < kBMax; ++k) {
          const int o = base + so.d[0][k][1] * kTW + so.d[0][k][0];
          sp = fma(dv.b_coef[k][1], X[1][o], fma(dv.b_coef[k][0], X[0][o], sp));
        }
        const int64_t q = (int64_t)pj * (a.n + 1) + pi;
        const int64_t o2 = 2 * (int64_t)a.L2;
        const T val = q == 0 ? pp_x : -sp;
        if (a.ms_s) {
          const T sc = (T)*a.ms_s, cc = (T)*a.ms_c;
          T yv = sc * val;
          if (cc != T(0)) yv += cc * pp_r1;
          const T vv = sc * pp_x;
          a.ms_r1y[o2 + q] = yv;
          a.ms_v[o2 + q] = vv;
          ms_acc += (double)vv * (double)yv;
        } else {
          a.y[o2 + q] = val;
        }
      }
    }
    if (a.ms_s) {   // the block's part of v . y (fixed order: deterministic)
      __shared__ double red[256 / kWave];
      const double wsum = wave_sum(ms_acc);
      if (tid % kWave == 0) red[tid / kWave] = wsum;
      __syncthreads();
      if (tid == 0) {
        double b = 0.0;
        for (int k = 0; k < 256 / kWave; ++k) b += red[k];
        a.ms_part[t] = b;
      }
    }
  }
}

template <typename T, int MODE>
static void launch_tiles(int n, const StencilArgs<T> &a, hipStream_t s, int K) {
  const int L = 2 * n + 1;
  const int tx = (L + kTileC - 1) / kTileC, ty = (L + kTileR - 1) / kTileR;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  FSI_REQUIRE(K >= 1 && K <= 65535, FSI_E_ARG, "lane count out of range");
  hipLaunchKernelGGL((k_stencil<T, MODE>), dim3((unsigned)(band * kXcd), (unsigned)K), dim3(256), 0, s, a, tx,
                     tiles, band);
  FSI_CHECK_LAUNCH();
}

// One lane stride for the vectors of a launch (null views take any)
static int64_t common_stride(std::initializer_list<std::pair<const void *, int64_t>> v, int K) {
  int64_t s = -1;
  for (const auto &e : v) {
    if (!e.first) continue;
    if (s < 0) s = e.second;
    FSI_REQUIRE(K == 1 || e.second == s, FSI_E_ARG, "lane views of one launch need one stride");
  }
  return s < 0 ? 0 : s;
}

template <typename T, int MODE>
void stencil_launch(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c1,
                    T c2, hipStream_t s, int K) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  static_assert(kTileR * kWave == 256 && 2 * kWave == kTileC, "one tile row per wave, two nodes per lane");
  const int64_t lv = common_stride({{x.p, x.s}, {b.p, b.s}, {d.p, d.s}, {y.p, y.s}}, K);
  StencilArgs<T> a{n, tab, x.p, b.p, d.p, y.p, (2 * n + 1) * (2 * n + 1), c1, c2, nullptr, nullptr, nullptr,
                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, lv, 0, 0};
  launch_tiles<T, MODE>(n, a, s, K);
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
                   xl ? xl + Ns : nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
  launch_tiles<T, SP_A11>(n, a, s, 1);
}

int stencil_a11_minres(int n, const StencilTable<double> *tab, const DivTable<double> *dv, LP<const double> x,
                       LP<double> v, LP<double> r1y, LP<const double> s_dev, LP<const double> c_dev,
                       LP<const double> slot_dev, int64_t vs, int nslot, LP<double> part, hipStream_t s, int K) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  FSI_REQUIRE(slot_dev.p && nslot >= 1, FSI_E_ARG, "the Lanczos block needs a slot index and at least one slot");
  const int L = 2 * n + 1, L2 = L * L;
  const int64_t lv = common_stride({{x.p, x.s}, {v.p, v.s}, {r1y.p, r1y.s}}, K);
  const int64_t ls = common_stride({{s_dev.p, s_dev.s}, {c_dev.p, c_dev.s}, {slot_dev.p, slot_dev.s}}, K);
  StencilArgs<double> a{n, tab, x.p, nullptr, nullptr, nullptr, L2, 0.0, 0.0, dv, nullptr, nullptr, nullptr, nullptr,
                        nullptr, s_dev.p, c_dev.p, v.p, r1y.p, part.p, lv, ls, part.s, slot_dev.p, vs, nslot};
  launch_tiles<double, SP_A11>(n, a, s, K);
  const int tx = (L + kTileC - 1) / kTileC, ty = (L + kTileR - 1) / kTileR;
  return tx * ty;
}

int stencil_tile_count(int n) {
  const int L = 2 * n + 1;
  return ((L + kTileC - 1) / kTileC) * ((L + kTileR - 1) / kTileR);
}
template void stencil_fluid_rows<double>(int, const StencilTable<double> *, const DivTable<double> *,
                                         const double *, double *, const int *, const int *, const double *,
                                         const double *, int64_t, hipStream_t);
template void stencil_fluid_rows<float>(int, const StencilTable<float> *, const DivTable<float> *, const float *,
                                        float *, const int *, const int *, const float *, const float *, int64_t,
                                        hipStream_t);

// ---------------------------------------------------------------- two steps per launch
// Temporal blocking of the Chebyshev smoother: two steps on a tile of kC2R x kC2W nodes.
// x is staged with a halo of four nodes (X0), the first step is computed on the tile plus
// a halo of two (X1, and its direction D1 on the tile), the second on the tile.  Dirichlet
// and out-of-lattice values are stored as 0 in X0 and X1 (zero columns); Dirichlet rows
// (identity) are stepped pointwise from global memory.  b and d are read where needed
// (pointwise).  Modes:
//   C2_PRE : the first step from x = 0 (x = d = s D^{-1} b) and two more: the whole
//            pre-smoothing of a degree-3 smoother; reads b, writes x and d.
//   C2_POST: two steps from x with the first direction coefficient c1 = 0 (no d read):
//            the start of the post-smoothing; reads x and b, writes y and d.
// Bytes per node: C2_PRE 6 w for three steps, C2_POST 8 w for two (w = value size,
// two components).
constexpr int kC2W = 124, kC2R = 8;                 // output tile (kC2W + 4 = 2 x 64 lanes)
constexpr int kC2W0 = kC2W + 8;                     // width of x with a halo of 4
constexpr int kC2W1 = kC2W + 4;                     // width of the first step (halo of 2)
static_assert(kC2W1 == 2 * kWave && kC2W0 == kTW, "lane layout and LDS offsets of the tables");

template <typename T>
struct Cheb2Args {
  int n;
  const StencilTable<T> *tab;
  const T *x, *b;
  T *d, *y;
  int L2;
  T s;                   // C2_PRE: scale of the first step
  T c1a, c2a, c1b, c2b;  // the two stencil steps
  int64_t lv;            // lane stride of x, b, d, y (lane = blockIdx.y)
};

// The staged tiles are stored as two planes of even and odd lattice columns
// (X[component][parity][row][column / 2]), so a half-wave pass over nodes of one parity
// reads consecutive words (no LDS bank conflicts).  Node at plane column h of parity PAR
// (= CLS & 1), neighbour (dI, dJ): parity (PAR + dI) & 1, plane column h + ((PAR + dI) >> 1).
template <typename T, int CLS, int ROWS, int HW, int NR>
__device__ __forceinline__ void split_products(const StencilTable<T> &tb, const T *X, const int (&row)[NR], int h,
                                               T (&s)[NR][2]) {
  constexpr int PAR = CLS & 1;
  constexpr int COMP = 2 * ROWS * HW;   // offset of the second component
  constexpr StencilOffsets so = stencil_offsets();
  constexpr CrossZero cz = cross_zero();
#pragma unroll
  for (int q = 0; q < NR; ++q) s[q][0] = s[q][1] = 0;
#pragma unroll
  for (int k = 0; k < kStencilCount[CLS]; ++k) {
    const int dI = so.d[CLS][k][0], dJ = so.d[CLS][k][1];
    const int off = (((PAR + dI) & 1) * ROWS + dJ) * HW + ((PAR + dI) >> 1);
    const T c0 = tb.coef[CLS][k][0], c1 = tb.coef[CLS][k][1], c2 = tb.coef[CLS][k][2], c3 = tb.coef[CLS][k][3];
#pragma unroll
    for (int q = 0; q < NR; ++q) {   // FMA chains: two FMAs per coefficient pair
      const int o = row[q] * HW + h + off;
      const T y0 = X[o], y1 = X[COMP + o];
      if (cz.z[CLS][k]) {   // xy = yx = 0 (fma with a zero coefficient adds nothing)
        s[q][0] = fma(c0, y0, s[q][0]);
        s[q][1] = fma(c3, y1, s[q][1]);
      } else {
        s[q][0] = fma(c1, y1, fma(c0, y0, s[q][0]));
        s[q][1] = fma(c3, y1, fma(c2, y0, s[q][1]));
      }
    }
  }
}

// rows of one parity class (the class is uniform over the wave: jodd is wave-uniform)
template <typename T, int PAR, int ROWS, int HW, int NR>
__device__ __forceinline__ void class_products(const StencilTable<T> &tb, int jodd, const T *X,
                                               const int (&row)[NR], int h, T (&s)[NR][2]) {
  if (jodd) split_products<T, PAR | 2, ROWS, HW, NR>(tb, X, row, h, s);
  else split_products<T, PAR, ROWS, HW, NR>(tb, X, row, h, s);
}

enum { C2_PRE = 0, C2_POST = 1 };

// A block of 64 RR threads owns a tile of RR rows.  Wave w owns region-1 row w + 2 (tile
// row w) and, for w < 4, one halo row (0, 1, RR + 2 or RR + 3) of the same parity; its
// lanes hold the nodes i = 2 lane + par of those rows (region-1 column i = tile column
// i - 2), so the tile row's b and first-step direction stay in registers for the second
// step.  All b loads are issued before x is staged.
template <typename T, int M, int RR>
__global__ void __launch_bounds__(64 * RR, 4) k_cheb2(Cheb2Args<T> a0, int tiles_x, int tiles, int band) {
  constexpr int NT = 64 * RR;                       // threads
  constexpr int kC2H0 = RR + 8, kC2H1 = RR + 4;     // rows of the staged x and the first step
  static_assert(RR >= 4 && RR % 2 == 0, "four halo rows go to the first four waves");
  constexpr int HW0 = kC2W0 / 2, HW1 = kC2W1 / 2;   // plane widths
  static_assert(kC2H1 * HW1 <= kC2H0 * HW0, "the first-step tile fits in the staged x");
  __shared__ T X0[2 * 2 * kC2H0 * HW0];             // [component][parity][row][column / 2]
  T *const X1 = X0;   // the first-step tile replaces x once every wave has read it
  const int t = (blockIdx.x % kXcd) * band + blockIdx.x / kXcd;
  if (t >= tiles) return;
  Cheb2Args<T> a = a0;
  lane_shift(a.x, a.lv);
  lane_shift(a.b, a.lv);
  lane_shift(a.d, a.lv);
  lane_shift(a.y, a.lv);
  const int n2 = 2 * a.n, L = n2 + 1;
  const int64_t N = a.L2;
  const int I0 = (t % tiles_x) * kC2W, J0 = (t / tiles_x) * RR;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const StencilTable<T> &tb = *a.tab;
  const bool halo = w < 4;                          // wave-uniform
  const int rows[2] = {w < 2 ? w : RR + w, w + 2};  // halo row (w < 4), tile row (region-1 rows)
  auto inside = [&](int I, int J) { return I > 0 && J > 0 && I < n2 && J < n2; };
  // b at the wave's region-1 nodes (0 outside the lattice)
  T bv[2][2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int J = J0 - 2 + rows[q];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int I = I0 - 2 + 2 * lane + par;
      bv[q][par][0] = 0;
      bv[q][par][1] = 0;
      if ((q == 1 || halo) && I >= 0 && J >= 0 && I <= n2 && J <= n2) {
        const int64_t r = (int64_t)J * L + I;
        bv[q][par][0] = a.b[r];
        bv[q][par][1] = a.b[N + r];
      }
    }
  }
  // phase A: x (or, from zero, the first step s D^{-1} b) with a halo of 4; all loads are
  // issued before the first LDS store
  constexpr int NE = kC2H0 * kC2W0, IT = (NE + NT - 1) / NT;
  T v[IT][2];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / kC2W0, tc = e % kC2W0;
    const int I = I0 - 4 + tc, J = J0 - 4 + tr;
    v[q][0] = 0;
    v[q][1] = 0;
    if (e < NE && inside(I, J)) {
      const int64_t r = (int64_t)J * L + I;
      v[q][0] = M == C2_PRE ? a.b[r] : a.x[r];
      v[q][1] = M == C2_PRE ? a.b[N + r] : a.x[N + r];
    }
  }
  if constexpr (M == C2_PRE) {
    // class-wise D^{-1} (scalar loads) picked per node: parity of I = parity of tc, of J = of tr
    T dv[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) dv[c][k] = tb.dinv[c][k];
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + NT * q, tr = e / kC2W0, tc = e % kC2W0;
      const int c = (tc & 1) | ((tr & 1) << 1);
      T di[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        di[k] = c == 0 ? dv[0][k] : c == 1 ? dv[1][k] : c == 2 ? dv[2][k] : dv[3][k];
      const T b0 = v[q][0], b1 = v[q][1];
      v[q][0] = a.s * (di[0] * b0 + di[1] * b1);
      v[q][1] = a.s * (di[2] * b0 + di[3] * b1);
    }
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / kC2W0, tc = e % kC2W0;
    if (e < NE) {
      const int o = ((tc & 1) * kC2H0 + tr) * HW0 + (tc >> 1);
      X0[o] = v[q][0];
      X0[2 * kC2H0 * HW0 + o] = v[q][1];
    }
  }
  __syncthreads();
  // phase B: first stencil step on the tile plus a halo of 2; a wave's rows have the same
  // parity, so one pass per column parity covers them with one set of coefficients
  T d1[2][2] = {{0, 0}, {0, 0}};   // tile row
  T x1v[2][2][2] = {};             // first-step values of the wave's rows
  const int jodd = __builtin_amdgcn_readfirstlane((J0 - 2 + rows[1]) & 1);
  auto phase_b = [&](auto q0_tag) {
    constexpr int Q0 = decltype(q0_tag)::value, NR = 2 - Q0;   // rows Q0..1
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int i = 2 * lane + par, I = I0 - 2 + i;   // I0 is even: I has the parity of i
      const int cls = par | (jodd << 1);
      int xr[NR];                                      // X0 rows; X0 column i + 2 = 2 (lane + 1) + par
#pragma unroll
      for (int k = 0; k < NR; ++k) xr[k] = rows[Q0 + k] + 2;
      T sp[NR][2];
      if (par) class_products<T, 1, kC2H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
      else class_products<T, 0, kC2H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
      const T *di = tb.dinv[cls];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int q = Q0 + k, row = rows[q], J = J0 - 2 + row;
        T &x10 = x1v[q][par][0], &x11 = x1v[q][par][1];
        x10 = 0;
        x11 = 0;
        if (inside(I, J)) {
          const int c0 = (par * kC2H0 + row + 2) * HW0 + lane + 1;
          const T x00 = X0[c0], x01 = X0[2 * kC2H0 * HW0 + c0];
          const T r0 = bv[q][par][0] - sp[k][0], r1 = bv[q][par][1] - sp[k][1];
          const T z0 = di[0] * r0 + di[1] * r1, z1 = di[2] * r0 + di[3] * r1;
          T e0, e1;
          if constexpr (M == C2_PRE) {   // d = x after the first step from zero
            e0 = a.c1a * x00 + a.c2a * z0;
            e1 = a.c1a * x01 + a.c2a * z1;
          } else {
            e0 = a.c2a * z0;
            e1 = a.c2a * z1;
          }
          x10 = x00 + e0;
          x11 = x01 + e1;
          if (q == 1) {
            d1[par][0] = e0;
            d1[par][1] = e1;
          }
        }
      }
    }
  };
  if (halo) phase_b(std::integral_constant<int, 0>{});
  else phase_b(std::integral_constant<int, 1>{});
  __syncthreads();   // every wave has read x: the first-step tile goes over it
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      if (q == 0 && !halo) continue;
      const int o1 = (par * kC2H1 + rows[q]) * HW1 + lane;   // column i = 2 lane + par
      X1[o1] = x1v[q][par][0];
      X1[2 * kC2H1 * HW1 + o1] = x1v[q][par][1];
    }
  __syncthreads();
  // phase C: second step on the tile row
  {
    const int row = rows[1], J = J0 - 2 + row;
    if (J <= n2) {
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const int i = 2 * lane + par, I = I0 - 2 + i;
        if (i < 2 || i >= 2 + kC2W || I > n2) continue;
        const int64_t r = (int64_t)J * L + I;
        const T b0 = bv[1][par][0], b1 = bv[1][par][1];
        T x20, x21, d20, d21;
        if (inside(I, J)) {
          const int cls = par | (jodd << 1);
          const int xr[1] = {row};
          T sp[1][2];
          if (par) class_products<T, 1, kC2H1, HW1, 1>(tb, jodd, X1, xr, lane, sp);
          else class_products<T, 0, kC2H1, HW1, 1>(tb, jodd, X1, xr, lane, sp);
          const T s0 = sp[0][0], s1 = sp[0][1];
          const int c1 = (par * kC2H1 + row) * HW1 + lane;
          const T r0 = b0 - s0, r1 = b1 - s1;
          const T *di = tb.dinv[cls];
          const T z0 = di[0] * r0 + di[1] * r1, z1 = di[2] * r0 + di[3] * r1;
          d20 = a.c1b * d1[par][0] + a.c2b * z0;
          d21 = a.c1b * d1[par][1] + a.c2b * z1;
          x20 = X1[c1] + d20;
          x21 = X1[2 * kC2H1 * HW1 + c1] + d21;
        } else {   // Dirichlet row: the identity, stepped pointwise
          T x00, x01, d00, d01;
          if constexpr (M == C2_PRE) {
            x00 = a.s * b0;
            x01 = a.s * b1;
            d00 = x00;
            d01 = x01;
          } else {
            x00 = a.x[r];
            x01 = a.x[N + r];
            d00 = 0;
            d01 = 0;
          }
          const T e0 = a.c1a * d00 + a.c2a * (b0 - x00), e1 = a.c1a * d01 + a.c2a * (b1 - x01);
          const T x10 = x00 + e0, x11 = x01 + e1;
          d20 = a.c1b * e0 + a.c2b * (b0 - x10);
          d21 = a.c1b * e1 + a.c2b * (b1 - x11);
          x20 = x10 + d20;
          x21 = x11 + d21;
        }
        if (a.d) {   // null when no later step reads the direction
          a.d[r] = d20;
          a.d[N + r] = d21;
        }
        a.y[r] = x20;
        a.y[N + r] = x21;
      }
    }
  }
}

// ---------------------------------------------------------------- three steps per launch
// The whole post-smoothing of a degree-3 smoother: from x, a step with c1 = 0 (c2a) and two
// steps (c1b, c2b), (c1c, c2c); reads x and b, writes y and d (8 w per node, as C2_POST).
// Tile of kC3R rows x kC3W nodes; x staged with a halo of 6 (X0), the first step on the tile
// plus a halo of 4 (region 1: kC3R + 8 rows x 128 nodes, X1 over X0), the second on the tile
// plus a halo of 2 (stored in region-1 coordinates, X2 over X1), the third on the tile.
// Every phase uses the lane layout of region 1 (lane holds columns i = 2 lane + par), so a
// thread's b and directions stay in registers from one step to the next.  Waves: wave w owns
// tile row w + 4 of region 1 in every phase and, for w < 8, one halo row: the inner halo rows
// 2, 3, R + 4, R + 5 (steps 1 and 2) go to waves 0-3, the outer halo rows 0, 1, R + 6, R + 7
// (step 1 only) to waves 4-7.
// With a coarse correction xc (the V-cycle's post-smoothing), the smoothing starts from
// x + P xc: the coarse nodes under the staged region go to LDS first and every staged
// interior node adds the coarse quadratic evaluated there (Sec. 4 multigrid transfer: the
// P2 interpolation of the coarse lattice, the same sums as the separate prolongation).
constexpr int kC3W = 120, kC3R = 8;
static_assert(kC3W + 8 == 2 * kWave && kC3W + 12 == kC2W0, "region-1 lane layout and staged width");

template <typename T, typename TY>
struct Cheb3Args {   // y stored as TY (the mixed form writes FP32 results into an FP64 vector)
  int n;
  const StencilTable<T> *tab;
  const T *x, *b;
  T *d;
  TY *y;
  int L2;
  T c2a, c1b, c2b, c1c, c2c;
  int64_t lv;    // lane stride of x, b, d, y (lane = blockIdx.y)
  const T *xc;   // coarse correction (lattice n / 2, two components) or null
  int64_t lc;    // its lane stride
  double *dot;   // per-tile sums of b . y over the tile's nodes (FP64), or null
  int64_t ldot;  // their lane stride
  const double *b64;   // with dot: the FP64 right-hand side the sums use instead of b, or null
  int64_t lb64;        // its lane stride
};

// Coarse P2 interpolation at an interior fine node (I, J) of the cell (I >> 2, J >> 2) at
// local position (A, B) = (I mod 4, J mod 4): the six P2 basis functions of the cell's
// triangle (lower right when A >= B, upper left otherwise) at (A / 4, B / 4); basis values
// are multiples of 1/8, exact in float.  XC holds the coarse nodes of the staged region
// ([row][column][component], row stride CW, origin (Ic0, Jc0) in coarse coordinates; 0 at
// Dirichlet nodes).  Sums in the order vertices 0, 1, 2, then edges 01, 12, 20.
template <typename T, int CW>
__device__ __forceinline__ void prolong_lds(const T *XC, int I, int J, int Ic0, int Jc0, T &s0, T &s1) {
  const int A = I & 3, B = J & 3;
  const int base = (2 * (J >> 2) - Jc0) * CW + 2 * (I >> 2) - Ic0;
  const bool lo = A >= B;
  const float xi = 0.25f * (float)A, eta = 0.25f * (float)B;
  const float l0 = lo ? 1.0f - xi : 1.0f - eta, l1 = lo ? xi - eta : xi, l2 = lo ? eta : eta - xi;
  const float phi[6] = {l0 * (2.0f * l0 - 1.0f), l1 * (2.0f * l1 - 1.0f), l2 * (2.0f * l2 - 1.0f),
                        4.0f * l0 * l1,         4.0f * l1 * l2,         4.0f * l2 * l0};
  const int off[6] = {0,
                      lo ? 2 : 2 * CW + 2,
                      lo ? 2 * CW + 2 : 2 * CW,
                      lo ? 1 : CW + 1,
                      lo ? CW + 2 : 2 * CW + 1,
                      CW + (lo ? 1 : 0)};
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const T w = (T)phi[q];
    const int o = 2 * (base + off[q]);
    s0 = fma(w, XC[o], s0);
    s1 = fma(w, XC[o + 1], s1);
  }
}

template <typename T, int RR, typename TY, bool PROL, bool DOT>
__global__ void __launch_bounds__(64 * RR, 4) k_cheb3(Cheb3Args<T, TY> a0, int tiles_x, int tiles, int band) {
  constexpr int NT = 64 * RR;
  constexpr int H0 = RR + 12, H1 = RR + 8;           // rows of the staged x and of region 1
  constexpr int W0 = kC3W + 12, HW0 = W0 / 2, HW1 = kWave;
  static_assert(RR >= 8 && RR % 2 == 0, "eight halo rows go to the first eight waves");
  static_assert(2 * H1 * HW1 <= 2 * H0 * HW0, "region 1 fits in the staged x");
  __shared__ T X0[2 * 2 * H0 * HW0];                 // [component][parity][row][column / 2]
  T *const X1 = X0;                                  // region-1 layout, rows H1, width 128
  const int t = (blockIdx.x % kXcd) * band + blockIdx.x / kXcd;
  if (t >= tiles) return;
  Cheb3Args<T, TY> a = a0;
  lane_shift(a.x, a.lv);
  lane_shift(a.b, a.lv);
  lane_shift(a.d, a.lv);
  lane_shift(a.y, a.lv);
  lane_shift(a.xc, a.lc);
  lane_shift(a.dot, a.ldot);
  lane_shift(a.b64, a.lb64);
  const int n2 = 2 * a.n, L = n2 + 1;
  const int64_t N = a.L2;
  const int I0 = (t % tiles_x) * kC3W, J0 = (t / tiles_x) * RR;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const StencilTable<T> &tb = *a.tab;
  const bool inner = w < 4, has_h = w < 8;          // wave-uniform
  // region-1 rows (origin J0 - 4): tile row, halo row
  const int rows[2] = {w + 4, inner ? (w < 2 ? 2 + w : RR + 2 + w) : (w < 6 ? w - 4 : RR + w)};
  auto inside = [&](int I, int J) { return I > 0 && J > 0 && I < n2 && J < n2; };
  // b at the wave's nodes (0 outside the lattice)
  T bv[2][2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int J = J0 - 4 + rows[q];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int I = I0 - 4 + 2 * lane + par;
      bv[q][par][0] = 0;
      bv[q][par][1] = 0;
      if ((q == 0 || has_h) && I >= 0 && J >= 0 && I <= n2 && J <= n2) {
        const int64_t r = (int64_t)J * L + I;
        bv[q][par][0] = a.b[r];
        bv[q][par][1] = a.b[N + r];
      }
    }
  }
  // coarse nodes under the staged region: coarse columns I0 / 2 - 4 .. I0 / 2 + W0 / 2 + 2,
  // rows J0 / 2 - 4 .. J0 / 2 + RR + 4 (the cells of fine columns I0 - 6 .. I0 + W0 - 7)
  constexpr int CW = 2 * ((W0 - 7) / 4) + 7, CH = 2 * ((RR + 5) / 4) + 7;
  static_assert(RR % 4 == 0 && kC3W % 4 == 0, "tile origins on coarse cell corners");
  __shared__ T XC[PROL ? 2 * CH * CW : 1];
  const int Ic0 = I0 / 2 - 4, Jc0 = J0 / 2 - 4;
  constexpr int NC = CH * CW, ITC = PROL ? (NC + NT - 1) / NT : 0;
  T cv[ITC > 0 ? ITC : 1][2];
  if constexpr (PROL) {   // loads issued before those of x; stored once they are in flight
    const int Lc = a.n + 1, nc2 = a.n;   // coarse lattice: 2 (n / 2) + 1 nodes a side
    const int64_t Nc = (int64_t)Lc * Lc;
#pragma unroll
    for (int q = 0; q < ITC; ++q) {
      const int e = tid + NT * q, Ic = Ic0 + e % CW, Jc = Jc0 + e / CW;
      cv[q][0] = 0;
      cv[q][1] = 0;
      if (e < NC && Ic > 0 && Jc > 0 && Ic < nc2 && Jc < nc2) {
        const int64_t k = (int64_t)Jc * Lc + Ic;
        cv[q][0] = a.xc[k];
        cv[q][1] = a.xc[Nc + k];
      }
    }
  }
  // stage x with a halo of 6 (0 at Dirichlet nodes and outside the lattice)
  constexpr int NE = H0 * W0, IT = (NE + NT - 1) / NT;
  T v[IT][2];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / W0, tc = e % W0;
    const int I = I0 - 6 + tc, J = J0 - 6 + tr;
    v[q][0] = 0;
    v[q][1] = 0;
    if (e < NE && inside(I, J)) {
      const int64_t r = (int64_t)J * L + I;
      v[q][0] = a.x[r];
      v[q][1] = a.x[N + r];
    }
  }
  if constexpr (PROL) {
#pragma unroll
    for (int q = 0; q < ITC; ++q) {
      const int e = tid + NT * q;
      if (e < NC) {
        XC[2 * e] = cv[q][0];
        XC[2 * e + 1] = cv[q][1];
      }
    }
    __syncthreads();   // the coarse nodes are in XC
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / W0, tc = e % W0;
    if (e < NE) {
      if constexpr (PROL) {
        const int I = I0 - 6 + tc, J = J0 - 6 + tr;
        if (inside(I, J)) {
          T s0, s1;
          prolong_lds<T, CW>(XC, I, J, Ic0, Jc0, s0, s1);
          v[q][0] += s0;
          v[q][1] += s1;
        }
      }
      const int o = ((tc & 1) * H0 + tr) * HW0 + (tc >> 1);
      X0[o] = v[q][0];
      X0[2 * H0 * HW0 + o] = v[q][1];
    }
  }
  __syncthreads();
  // a wave's rows have one parity: the class is wave-uniform per column parity
  const int jodd = __builtin_amdgcn_readfirstlane((J0 - 4 + rows[0]) & 1);
  // step 1 on region 1 (from X0), c1 = 0
  T d1[2][2][2] = {};   // [row][par][component]
  T xs[2][2][2] = {};   // values of the step, stored after the barrier
  auto step1 = [&](auto nr_tag) {
    constexpr int NR = decltype(nr_tag)::value;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int I = I0 - 4 + 2 * lane + par;
      const int cls = par | (jodd << 1);
      int xr[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) xr[k] = rows[k] + 2;
      T sp[NR][2];
      if (par) class_products<T, 1, H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
      else class_products<T, 0, H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
      const T *di = tb.dinv[cls];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int J = J0 - 4 + rows[k];
        if (inside(I, J)) {
          const int c0 = (par * H0 + rows[k] + 2) * HW0 + lane + 1;
          const T x00 = X0[c0], x01 = X0[2 * H0 * HW0 + c0];
          const T r0 = bv[k][par][0] - sp[k][0], r1 = bv[k][par][1] - sp[k][1];
          const T e0 = a.c2a * (di[0] * r0 + di[1] * r1), e1 = a.c2a * (di[2] * r0 + di[3] * r1);
          d1[k][par][0] = e0;
          d1[k][par][1] = e1;
          xs[k][par][0] = x00 + e0;
          xs[k][par][1] = x01 + e1;
        }
      }
    }
  };
  if (has_h) step1(std::integral_constant<int, 2>{});
  else step1(std::integral_constant<int, 1>{});
  __syncthreads();   // every wave has read X0
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      if (q == 1 && !has_h) continue;
      const int o1 = (par * H1 + rows[q]) * HW1 + lane;
      X1[o1] = xs[q][par][0];
      X1[2 * H1 * HW1 + o1] = xs[q][par][1];
    }
  __syncthreads();
  // step 2 on region 2 (region-1 columns 2..125, rows 2..R+5): tile row, inner halo row
  T d2[2][2] = {};      // tile row only
  auto step2 = [&](auto nr_tag) {
    constexpr int NR = decltype(nr_tag)::value;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int i = 2 * lane + par, I = I0 - 4 + i;
      const int cls = par | (jodd << 1);
      int xr[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) xr[k] = rows[k];
      // lanes 0 and 63 hold no region-2 node: their (discarded) products read in-row columns
      const int h = lane < 1 ? 1 : lane > 62 ? 62 : lane;
      T sp[NR][2];
      if (par) class_products<T, 1, H1, HW1, NR>(tb, jodd, X1, xr, h, sp);
      else class_products<T, 0, H1, HW1, NR>(tb, jodd, X1, xr, h, sp);
      const T *di = tb.dinv[cls];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int J = J0 - 4 + rows[k];
        T x0 = 0, x1 = 0;
        if (i >= 2 && i < 2 + kC3W + 4 && inside(I, J)) {
          const int c1 = (par * H1 + rows[k]) * HW1 + lane;
          const T r0 = bv[k][par][0] - sp[k][0], r1 = bv[k][par][1] - sp[k][1];
          const T z0 = di[0] * r0 + di[1] * r1, z1 = di[2] * r0 + di[3] * r1;
          const T e0 = a.c1b * d1[k][par][0] + a.c2b * z0, e1 = a.c1b * d1[k][par][1] + a.c2b * z1;
          x0 = X1[c1] + e0;
          x1 = X1[2 * H1 * HW1 + c1] + e1;
          if (k == 0) {
            d2[par][0] = e0;
            d2[par][1] = e1;
          }
        }
        xs[k][par][0] = x0;
        xs[k][par][1] = x1;
      }
    }
  };
  if (inner) step2(std::integral_constant<int, 2>{});
  else step2(std::integral_constant<int, 1>{});
  __syncthreads();   // every wave has read X1
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      if (q == 1 && !inner) continue;
      const int o1 = (par * H1 + rows[q]) * HW1 + lane;
      X1[o1] = xs[q][par][0];
      X1[2 * H1 * HW1 + o1] = xs[q][par][1];
    }
  __syncthreads();
  // step 3 on the tile row (region-1 columns 4..R+3 of the tile: i in [4, 4 + kC3W))
  double by = 0.0;   // the thread's part of b . y
  {
    const int row = rows[0], J = J0 - 4 + row;
    if (J <= n2) {
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const int i = 2 * lane + par, I = I0 - 4 + i;
        if (i < 4 || i >= 4 + kC3W || I > n2) continue;
        const int64_t r = (int64_t)J * L + I;
        const T b0 = bv[0][par][0], b1 = bv[0][par][1];
        T y0, y1, e0, e1;
        if (inside(I, J)) {
          const int cls = par | (jodd << 1);
          const int xr[1] = {row};
          T sp[1][2];
          if (par) class_products<T, 1, H1, HW1, 1>(tb, jodd, X1, xr, lane, sp);
          else class_products<T, 0, H1, HW1, 1>(tb, jodd, X1, xr, lane, sp);
          const int c1 = (par * H1 + row) * HW1 + lane;
          const T r0 = b0 - sp[0][0], r1 = b1 - sp[0][1];
          const T *di = tb.dinv[cls];
          const T z0 = di[0] * r0 + di[1] * r1, z1 = di[2] * r0 + di[3] * r1;
          e0 = a.c1c * d2[par][0] + a.c2c * z0;
          e1 = a.c1c * d2[par][1] + a.c2c * z1;
          y0 = X1[c1] + e0;
          y1 = X1[2 * H1 * HW1 + c1] + e1;
        } else {   // Dirichlet row: the identity, stepped pointwise
          const T x00 = a.x[r], x01 = a.x[N + r];
          const T f0 = a.c2a * (b0 - x00), f1 = a.c2a * (b1 - x01);
          const T x10 = x00 + f0, x11 = x01 + f1;
          const T g0 = a.c1b * f0 + a.c2b * (b0 - x10), g1 = a.c1b * f1 + a.c2b * (b1 - x11);
          const T x20 = x10 + g0, x21 = x11 + g1;
          e0 = a.c1c * g0 + a.c2c * (b0 - x20);
          e1 = a.c1c * g1 + a.c2c * (b1 - x21);
          y0 = x20 + e0;
          y1 = x21 + e1;
        }
        if (a.d) {   // null when no later step reads the direction
          a.d[r] = e0;
          a.d[N + r] = e1;
        }
        a.y[r] = (TY)y0;
        a.y[N + r] = (TY)y1;
        if constexpr (DOT) {
          if constexpr (std::is_same<T, double>::value) {   // b is the FP64 right-hand side
            by += (double)b0 * (double)(TY)y0 + (double)b1 * (double)(TY)y1;
          } else {
            const double f0 = a.b64 ? a.b64[r] : (double)b0, f1 = a.b64 ? a.b64[N + r] : (double)b1;
            by += f0 * (double)(TY)y0 + f1 * (double)(TY)y1;
          }
        }
      }
    }
  }
  if constexpr (DOT) {   // the tile's sum in a fixed order: lanes by shuffles, then waves
    __shared__ double red[RR];
    by = wave_sum(by);
    if (lane == 0) red[w] = by;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < RR; ++k) s += red[k];
      a.dot[t] = s;
    }
  }
}

int cheb3_dot_count(int n) {
  const int L = 2 * n + 1;
  return ((L + kC3W - 1) / kC3W) * ((L + kC3R - 1) / kC3R);
}

template <typename T, typename TY>
void cheb3_post(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<TY> y, T c2a, T c1b,
                T c2b, T c1c, T c2c, hipStream_t st, int K, LP<const T> xc, LP<double> dot,
                LP<const double> b64) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  FSI_REQUIRE(K >= 1 && K <= 65535, FSI_E_ARG, "lane count out of range");
  FSI_REQUIRE(!xc.p || (n % 2 == 0 && n >= 4), FSI_E_ARG, "a coarse correction needs an even fluid grid");
  FSI_REQUIRE(!xc.p || K == 1 || xc.s > 0, FSI_E_ARG, "lane views of the coarse correction need a stride");
  const int L = 2 * n + 1;
  const int tx = (L + kC3W - 1) / kC3W, ty = (L + kC3R - 1) / kC3R;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  const int64_t lv = common_stride({{x.p, x.s}, {b.p, b.s}, {d.p, d.s}, {y.p, y.s}}, K);
  FSI_REQUIRE(!dot.p || K == 1 || dot.s >= tiles, FSI_E_ARG, "lane stride of the tile sums too small");
  FSI_REQUIRE(!b64.p || (dot.p && (K == 1 || b64.s > 0) && !std::is_same<T, double>::value), FSI_E_ARG,
              "an FP64 right-hand side only for the sums of the FP32 form");
  Cheb3Args<T, TY> a{n, tab, x.p, b.p, d.p, y.p, L * L, c2a, c1b, c2b, c1c, c2c, lv, xc.p, xc.s, dot.p, dot.s,
                     b64.p, b64.s};
  const dim3 grid((unsigned)(band * kXcd), (unsigned)K), block(64 * kC3R);
  if (xc.p && dot.p)
    hipLaunchKernelGGL((k_cheb3<T, kC3R, TY, true, true>), grid, block, 0, st, a, tx, tiles, band);
  else if (xc.p)
    hipLaunchKernelGGL((k_cheb3<T, kC3R, TY, true, false>), grid, block, 0, st, a, tx, tiles, band);
  else if (dot.p)
    hipLaunchKernelGGL((k_cheb3<T, kC3R, TY, false, true>), grid, block, 0, st, a, tx, tiles, band);
  else
    hipLaunchKernelGGL((k_cheb3<T, kC3R, TY, false, false>), grid, block, 0, st, a, tx, tiles, band);
  FSI_CHECK_LAUNCH();
}
template void cheb3_post<double, double>(int, const StencilTable<double> *, LP<const double>, LP<const double>,
                                         LP<double>, LP<double>, double, double, double, double, double, hipStream_t,
                                         int, LP<const double>, LP<double>, LP<const double>);
template void cheb3_post<float, float>(int, const StencilTable<float> *, LP<const float>, LP<const float>, LP<float>,
                                       LP<float>, float, float, float, float, float, hipStream_t, int,
                                       LP<const float>, LP<double>, LP<const double>);
template void cheb3_post<float, double>(int, const StencilTable<float> *, LP<const float>, LP<const float>,
                                        LP<float>, LP<double>, float, float, float, float, float, hipStream_t, int,
                                        LP<const float>, LP<double>, LP<const double>);

template <typename T>
void cheb2_pre(int n, const StencilTable<T> *tab, LP<const T> b, LP<T> d, LP<T> x, T s, T c1a, T c2a, T c1b,
               T c2b, hipStream_t st, int K) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  FSI_REQUIRE(K >= 1 && K <= 65535, FSI_E_ARG, "lane count out of range");
  const int L = 2 * n + 1;
  const int tx = (L + kC2W - 1) / kC2W, ty = (L + kC2R - 1) / kC2R;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  const int64_t lv = common_stride({{b.p, b.s}, {d.p, d.s}, {x.p, x.s}}, K);
  Cheb2Args<T> a{n, tab, nullptr, b.p, d.p, x.p, L * L, s, c1a, c2a, c1b, c2b, lv};
  hipLaunchKernelGGL((k_cheb2<T, C2_PRE, kC2R>), dim3((unsigned)(band * kXcd), (unsigned)K), dim3(64 * kC2R), 0,
                     st, a, tx, tiles, band);
  FSI_CHECK_LAUNCH();
}

template <typename T>
void cheb2_post(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c2a, T c1b,
                T c2b, hipStream_t st, int K) {
  FSI_REQUIRE((int64_t)(2 * n + 1) * (2 * n + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  FSI_REQUIRE(K >= 1 && K <= 65535, FSI_E_ARG, "lane count out of range");
  const int L = 2 * n + 1;
  const int tx = (L + kC2W - 1) / kC2W, ty = (L + kC2R - 1) / kC2R;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  const int64_t lv = common_stride({{x.p, x.s}, {b.p, b.s}, {d.p, d.s}, {y.p, y.s}}, K);
  Cheb2Args<T> a{n, tab, x.p, b.p, d.p, y.p, L * L, T(0), T(0), c2a, c1b, c2b, lv};
  hipLaunchKernelGGL((k_cheb2<T, C2_POST, kC2R>), dim3((unsigned)(band * kXcd), (unsigned)K), dim3(64 * kC2R), 0,
                     st, a, tx, tiles, band);
  FSI_CHECK_LAUNCH();
}

#define FSI_CHEB2_INST(T)                                                                                   \
  template void cheb2_pre<T>(int, const StencilTable<T> *, LP<const T>, LP<T>, LP<T>, T, T, T, T, T,         \
                             hipStream_t, int);                                                             \
  template void cheb2_post<T>(int, const StencilTable<T> *, LP<const T>, LP<const T>, LP<T>, LP<T>, T, T, T, \
                              hipStream_t, int);
FSI_CHEB2_INST(double)
FSI_CHEB2_INST(float)
#undef FSI_CHEB2_INST

// ---------------------------------------------------------------- residual and restriction
// bc = R (b - A_f x) = P^T r for the multigrid descent (Sec. 4): the residual of the fine
// nodes under a coarse tile is computed from x staged in LDS and kept in LDS for the
// restriction sums, so r never goes to HBM (reads x and b, writes bc).  A block of 8 waves
// owns kRRr coarse rows x kRRc coarse columns; a coarse node (Ic, Jc) gathers the interior
// fine nodes within 3 of (2 Ic, 2 Jc), so the residual covers 2 kRRr + 5 fine rows and
// 2 kRRc + 5 columns (region origin (2 Ic0 - 4, 2 Jc0 - 4), lanes on columns 2 lane + par as
// in the smoothing kernels) and x is staged with 2 more on every side.  Restriction sums in
// the order of the restriction table; residual products in the order of the stencil table.
constexpr int kRRr = 8, kRRc = 60;
static_assert(2 * kRRc + 8 == 2 * kWave, "residual region fits the lane layout");

template <typename T>
struct ResidRestrArgs {
  int n;
  const StencilTable<T> *tab;
  const P2RestrTable<T> *rt;
  const T *x, *b;
  T *bc;
  int64_t lv, lc;   // lane strides of the fine (x, b) and coarse (bc) vectors
};

template <typename T>
__global__ void __launch_bounds__(512, 4) k_resid_restrict(ResidRestrArgs<T> a0, int tiles_x, int tiles, int band) {
  constexpr int NT = 512;
  constexpr int H1 = 2 * kRRr + 8;                   // residual region rows (1 .. H1 - 3 used)
  constexpr int H0 = H1 + 2, W0 = kC2W0, HW0 = W0 / 2;
  constexpr int RW = 2 * kWave;                      // residual region columns
  static_assert(kRRr == 8, "one coarse row per wave");
  __shared__ T X0[2 * 2 * H0 * HW0];                 // x: [component][parity][row][column / 2]
  T *const R = X0;                                   // then r: [component][row][column]
  static_assert(2 * H1 * RW <= 2 * 2 * H0 * HW0, "the residual fits over the staged x");
  const int t = (blockIdx.x % kXcd) * band + blockIdx.x / kXcd;
  if (t >= tiles) return;
  ResidRestrArgs<T> a = a0;
  lane_shift(a.x, a.lv);
  lane_shift(a.b, a.lv);
  lane_shift(a.bc, a.lc);
  const int n2 = 2 * a.n, L = n2 + 1, Lc = a.n + 1;
  const int64_t N = (int64_t)L * L, Nc = (int64_t)Lc * Lc;
  const int Ic0 = (t % tiles_x) * kRRc, Jc0 = (t / tiles_x) * kRRr;
  const int IR = 2 * Ic0 - 4, JR = 2 * Jc0 - 4;      // residual region origin (even)
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const StencilTable<T> &tb = *a.tab;
  auto inside = [&](int I, int J) { return I > 0 && J > 0 && I < n2 && J < n2; };
  // residual rows 1 + w, 9 + w, 17 + w (the third for waves 0-4): one parity per wave
  const bool three = w < 5;
  const int rows[3] = {1 + w, 9 + w, 17 + w};
  auto needed = [&](int i, int I, int J) { return i >= 1 && i < RW - 2 && inside(I, J); };
  T bv[3][2][2];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int J = JR + rows[q];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int i = 2 * lane + par, I = IR + i;
      bv[q][par][0] = 0;
      bv[q][par][1] = 0;
      if ((q < 2 || three) && needed(i, I, J)) {
        const int64_t r = (int64_t)J * L + I;
        bv[q][par][0] = a.b[r];
        bv[q][par][1] = a.b[N + r];
      }
    }
  }
  // stage x with a halo of 2 around the residual region (0 at Dirichlet nodes and outside)
  constexpr int NE = H0 * W0, IT = (NE + NT - 1) / NT;
  T v[IT][2];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / W0, tc = e % W0;
    const int I = IR - 2 + tc, J = JR - 2 + tr;
    v[q][0] = 0;
    v[q][1] = 0;
    if (e < NE && inside(I, J)) {
      const int64_t r = (int64_t)J * L + I;
      v[q][0] = a.x[r];
      v[q][1] = a.x[N + r];
    }
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + NT * q, tr = e / W0, tc = e % W0;
    if (e < NE) {
      const int o = ((tc & 1) * H0 + tr) * HW0 + (tc >> 1);
      X0[o] = v[q][0];
      X0[2 * H0 * HW0 + o] = v[q][1];
    }
  }
  __syncthreads();
  const int jodd = __builtin_amdgcn_readfirstlane((JR + rows[0]) & 1);
  // rows 0-1 of the wave together (one pass over the coefficients), then row 2
  auto resid = [&](auto q0_tag, auto nr_tag) {   // r over b (0 where not needed: b was not read)
    constexpr int Q0 = decltype(q0_tag)::value, NR = decltype(nr_tag)::value;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int i = 2 * lane + par, I = IR + i;
      int xr[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) xr[k] = rows[Q0 + k] + 2;
      T sp[NR][2];
      if (par) class_products<T, 1, H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
      else class_products<T, 0, H0, HW0, NR>(tb, jodd, X0, xr, lane + 1, sp);
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (needed(i, I, JR + rows[Q0 + k])) {
          bv[Q0 + k][par][0] -= sp[k][0];
          bv[Q0 + k][par][1] -= sp[k][1];
        }
    }
  };
  resid(std::integral_constant<int, 0>{}, std::integral_constant<int, 2>{});
  if (three) resid(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
  __syncthreads();   // every wave has read x: r goes over it
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q == 2 && !three) continue;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int o = rows[q] * RW + 2 * lane + par;
      R[o] = bv[q][par][0];
      R[H1 * RW + o] = bv[q][par][1];
    }
  }
  __syncthreads();
  // restriction: wave w owns coarse row Jc0 + w; lanes 0-29 the even columns, 32-61 the odd
  const int Jc = Jc0 + w, hi = lane >> 5, Ic = Ic0 + 2 * (lane & 31) + hi;
  if ((lane & 31) >= kRRc / 2 || Ic >= Lc || Jc >= Lc) return;
  T s0 = 0, s1 = 0;
  if (!(Ic == 0 || Jc == 0 || Ic == a.n || Jc == a.n)) {
    const P2RestrTable<T> &rt = *a.rt;
    constexpr RestrOffsets ro = restrict_offsets();
    const int c0 = (2 * w + 4) * RW + 2 * (Ic - Ic0) + 4;   // the coarse node's fine position
    auto gather = [&](auto cls_tag) {
      constexpr int CLS = decltype(cls_tag)::value;
#pragma unroll
      for (int k = 0; k < kRestrCount[CLS]; ++k) {
        const int o = c0 + ro.d[CLS][k][1] * RW + ro.d[CLS][k][0];
        const T wk = rt.w[CLS][k];
        s0 = fma(wk, R[o], s0);
        s1 = fma(wk, R[H1 * RW + o], s1);
      }
    };
    if (Jc & 1) {
      if (hi) gather(std::integral_constant<int, 3>{});
      else gather(std::integral_constant<int, 2>{});
    } else {
      if (hi) gather(std::integral_constant<int, 1>{});
      else gather(std::integral_constant<int, 0>{});
    }
  }
  const int64_t q = (int64_t)Jc * Lc + Ic;
  a.bc[q] = s0;
  a.bc[Nc + q] = s1;
}

template <typename T>
void resid_restrict(int nf, const StencilTable<T> *tab, const P2RestrTable<T> *rtab, LP<const T> x, LP<const T> b,
                    LP<T> bc, hipStream_t s, int K) {
  FSI_REQUIRE((int64_t)(2 * nf + 1) * (2 * nf + 1) < INT32_MAX, FSI_E_ARG, "grid too large for 32-bit stencil indices");
  FSI_REQUIRE(K >= 1 && K <= 65535, FSI_E_ARG, "lane count out of range");
  FSI_REQUIRE(nf % 2 == 0 && nf >= 4, FSI_E_ARG, "restriction needs an even fluid grid");
  FSI_REQUIRE(K == 1 || bc.s > 0, FSI_E_ARG, "lane views of the coarse vector need a stride");
  const int Lc = nf + 1;
  const int tx = (Lc + kRRc - 1) / kRRc, ty = (Lc + kRRr - 1) / kRRr;
  const int tiles = tx * ty, band = (tiles + kXcd - 1) / kXcd;
  const int64_t lv = common_stride({{x.p, x.s}, {b.p, b.s}}, K);
  ResidRestrArgs<T> a{nf, tab, rtab, x.p, b.p, bc.p, lv, bc.s};
  hipLaunchKernelGGL(k_resid_restrict<T>, dim3((unsigned)(band * kXcd), (unsigned)K), dim3(512), 0, s, a, tx, tiles,
                     band);
  FSI_CHECK_LAUNCH();
}
template void resid_restrict<double>(int, const StencilTable<double> *, const P2RestrTable<double> *,
                                     LP<const double>, LP<const double>, LP<double>, hipStream_t, int);
template void resid_restrict<float>(int, const StencilTable<float> *, const P2RestrTable<float> *, LP<const float>,
                                    LP<const float>, LP<float>, hipStream_t, int);

#define FSI_STENCIL_INST(T, M)                                                                              \
  template void stencil_launch<T, M>(int, const StencilTable<T> *, LP<const T>, LP<const T>, LP<T>, LP<T>, T, T, \
                                     hipStream_t, int);
FSI_STENCIL_INST(double, SP_APPLY)
FSI_STENCIL_INST(double, SP_RESID)
FSI_STENCIL_INST(double, SP_CHEB)
FSI_STENCIL_INST(float, SP_APPLY)
FSI_STENCIL_INST(float, SP_RESID)
FSI_STENCIL_INST(float, SP_CHEB)
#undef FSI_STENCIL_INST

}  // namespace fsi
