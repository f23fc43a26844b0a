// Block preconditioners (Sec. 5) and the outer Krylov solve (Sec. 6).
//
// P = diag(A11, A22) or [[A11, 0], [A21, A22]], applied exactly up to the inner tolerance:
//  * A22^{-1} in closed form: A22 = [[A_s, -C_s], [-(1/dt) C_s, 0]] gives
//      z_X = -dt C_s^{-1} r_lam,   z_lam = C_s^{-1} (A_s z_X - r_X),
//    with C_s^{-1} by Chebyshev iteration on D^{-1} C_s, whose spectrum lies in [1/2, 2] for
//    P1 triangles (Wathen's bound), run to the rounding level; always FP64 (the block is
//    small and its exactness matters);
//  * A11^{-1} by preconditioned MINRES on [[A_f, -B^T], [-B, pin]] to a relative tolerance,
//    with the SPD block preconditioner diag(V, S^{-1}):
//      V      one V-cycle of geometric multigrid for A_f on the nested P2 grids
//             (Chebyshev smoothing with 2x2 point-block Jacobi, exact coarse solve);
//      S^{-1} the Cahouet-Chabard approximation nu M_p^{-1} + (rho/dt) L_p^{-1} of the
//             pressure Schur complement, with M_p^{-1} by Chebyshev-Jacobi and L_p^{-1} by
//             one P1 multigrid V-cycle; the pinned node is the identity.
// The outer solve is right-preconditioned flexible GMRES(m) with classical Gram-Schmidt
// applied twice, FP64 Arnoldi vectors and the Givens reduction on the host.  Mixed
// precision (FP32) runs the preconditioner's multigrid and Schur parts in FP32; the
// FP32_IR variant also applies the operator in FP32 inside the Arnoldi process and wraps
// the cycles in iterative refinement on the FP64 residual.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "ctx.h"
#include "kernels.h"
#include "lattice.h"
#include "q2.h"
#include "stencil.h"

namespace fsi {

// FSI_TRACE=1 in the environment prints one line per inner solve and per outer cycle.
static bool trace_on() {
  static int on = -1;
  if (on < 0) {
    const char *e = std::getenv("FSI_TRACE");
    on = (e && e[0] == '1') ? 1 : 0;
  }
  return on == 1;
}

template <typename T>
void apply_a11(Ctx &c, const T *x, T *y);
// A11 on FP64 vectors with arithmetic (and matrix values) in TA
template <typename TA>
void apply_a11_on64(Ctx &c, const double *x, double *y);

// ---------------------------------------------------------------- small kernels
// First Chebyshev step from x = 0: d = x = scale * Dinv b (NC components of `nodes`).
template <typename T, int W, int NC>
__global__ void k_dinv_first(int64_t nodes, const T *dinv, const T *b, T scale, T *d, T *x) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nodes) return;
  if constexpr (W == 4) {
    T b0 = b[r], b1 = b[nodes + r];
    T z0 = scale * (dinv[4 * r] * b0 + dinv[4 * r + 1] * b1);
    T z1 = scale * (dinv[4 * r + 2] * b0 + dinv[4 * r + 3] * b1);
    d[r] = z0; x[r] = z0;
    d[nodes + r] = z1; x[nodes + r] = z1;
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T z = scale * dinv[r] * b[c * nodes + r];
      d[c * nodes + r] = z;
      x[c * nodes + r] = z;
    }
  }
}

// y = A x for a dense row-major m x m matrix (the coarsest multigrid level); lane
// blockIdx.y reads x and writes y at + lane m.  One wave per row, four rows per block; each
// lane loads VW consecutive entries at once (16 B when the row length and x allow it) and
// keeps 64 B of the row in flight (U loads), with a partial sum in double for each load.
template <typename T, int VW>
struct alignas(sizeof(T) * VW) DenseVec {
  T v[VW];
};
constexpr int kDenseRows = 4;
template <typename T, int VW>
__global__ void __launch_bounds__(kDenseRows * kWave) k_dense_mv(int m, const T *A, const T *x, T *y) {
  constexpr int U = 64 / (VW * (int)sizeof(T));
  const int lane = threadIdx.x % kWave;
  const int r = blockIdx.x * kDenseRows + threadIdx.x / kWave;
  if (r >= m) return;   // whole waves leave: the sums below stay within a wave
  x += (int64_t)blockIdx.y * m;
  y += (int64_t)blockIdx.y * m;
  using V = DenseVec<T, VW>;
  const V *a = reinterpret_cast<const V *>(A + (int64_t)r * m);
  const V *xv = reinterpret_cast<const V *>(x);
  const int mv = m / VW;
  double sum[U] = {};
  int k = lane;
  for (; k + (U - 1) * kWave < mv; k += U * kWave) {
    V av[U], xx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = a[k + u * kWave];
      xx[u] = xv[k + u * kWave];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < VW; ++c) sum[u] += (double)av[u].v[c] * (double)xx[u].v[c];
  }
  for (; k < mv; k += kWave) {
    const V a0 = a[k], x0 = xv[k];
#pragma unroll
    for (int c = 0; c < VW; ++c) sum[0] += (double)a0.v[c] * (double)x0.v[c];
  }
#pragma unroll
  for (int h = U / 2; h > 0; h /= 2)   // pairwise: the U = 4 order (s0 + s1) + (s2 + s3)
#pragma unroll
    for (int u = 0; u < h; ++u) sum[u] = sum[2 * u] + sum[2 * u + 1];
  const double s = wave_sum(sum[0]);
  if (lane == 0) y[r] = (T)s;
}

// the launch: the widest load the row length and the alignment of A and x allow
template <typename T>
static void dense_mv(int m, const T *A, const T *x, T *y, int K, hipStream_t s) {
  const dim3 grid((unsigned)((m + kDenseRows - 1) / kDenseRows), (unsigned)K), block(kDenseRows * kWave);
  auto fits = [&](int vw) {
    const uintptr_t b = sizeof(T) * vw;
    return m % vw == 0 && (uintptr_t)A % b == 0 && (uintptr_t)x % b == 0;
  };
  constexpr int W16 = 16 / (int)sizeof(T);
  if (fits(W16)) hipLaunchKernelGGL((k_dense_mv<T, W16>), grid, block, 0, s, m, A, x, y);
  else if (fits(2)) hipLaunchKernelGGL((k_dense_mv<T, 2>), grid, block, 0, s, m, A, x, y);
  else hipLaunchKernelGGL((k_dense_mv<T, 1>), grid, block, 0, s, m, A, x, y);
  FSI_CHECK_LAUNCH();
}

// y = a x + b y + c z
template <typename T>
__global__ void k_axpbypcz(T *y, const T *x, const T *z, T a, T b, T c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i] + c * z[i];
}

// y -= (alpha[0] * s) r   (alpha on the device)
template <typename T>
__global__ void k_sub_dev(T *y, const T *r, const double *alpha, double s, int64_t n) {
  T c = (T)(alpha[0] * s);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] -= c * r[i];
}

// MINRES direction and iterate: wn = (v - e w1 - d w2) / g;  x += phi wn
template <typename T>
__global__ void k_minres_update(T *wn, const T *v, const T *w1, const T *w2, T *x, T e, T d, T ginv,
                                T phi, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T w = (v[i] - e * w1[i] - d * w2[i]) * ginv;
    wn[i] = w;
    x[i] += phi * w;
  }
}

// The Schur approximation of the discontinuous pair on the pressure unknowns:
// z = nu M_p^{-1} r + (rho/dt) x_L (M_p diagonal, x_L the V-cycle on L = B D^{-1} B^T) in T, stored
// as TZ, except z[0] = r[0] rounded through T (the pinned unknown)
template <typename TZ, typename T>
__global__ void k_q_pres(TZ *z, const TZ *r, const T *xl, const T *mpinv, T nu, T rdt, int64_t np) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const T v = (T)r[i];
    z[i] = (TZ)(i == 0 ? v : nu * mpinv[i] * v + rdt * xl[i]);
  }
}

template <typename T>
__global__ void k_set_pinned(T *z, const T *r, int64_t ls) {   // lane blockIdx.y at + lane ls
  if (threadIdx.x == 0 && blockIdx.x == 0) z[(int64_t)blockIdx.y * ls] = r[(int64_t)blockIdx.y * ls];
}

// The pressure part of the A11 preconditioner's output with the dot product r . z of its
// entries: z = a x + b y computed in T and stored as TZ, except z[0] = r[0] rounded through T
// (pinned entry), and block k of kPresDotBlocks stores its part of sum r z (FP64, fixed
// partition and order) at part[k]; the sums take r64 in place of r when given (an FP32
// output of the mixed form, r its FP32 copy).  Lane blockIdx.y: z, r, r64 at + lane ls, x, y
// at + lane lx, part at + lane lp.
constexpr int kPresDotBlocks = 256;
// Parts of r . z from the pressure output: one per tile of the fused launch (matrix-free
// pressure hierarchy) or kPresDotBlocks; the slots per lane hold either
static int pres_dot_slots(int n) { return std::max(kPresDotBlocks, p1_multi_tiles(n)); }
static int pres_dot_count(const Ctx &c) { return c.mgp.stencil ? p1_multi_tiles(c.n) : kPresDotBlocks; }
template <typename TZ, typename T>
__global__ void __launch_bounds__(kRedBlock) k_pres_out_dot(TZ *z, const TZ *r, const T *x, const T *y, T a, T b,
                                                            int64_t n, int64_t ls, int64_t lx, double *part,
                                                            int64_t lp, const double *r64) {
  z += (int64_t)blockIdx.y * ls;
  r += (int64_t)blockIdx.y * ls;
  if (r64) r64 += (int64_t)blockIdx.y * ls;
  x += (int64_t)blockIdx.y * lx;
  y += (int64_t)blockIdx.y * lx;
  const int64_t chunk = (n + kPresDotBlocks - 1) / kPresDotBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kRedBlock) {
    const TZ v = (TZ)(i == 0 ? (T)r[0] : a * x[i] + b * y[i]);
    z[i] = v;
    s += (r64 ? r64[i] : (double)r[i]) * (double)v;
  }
  const double t = block_sum(s);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * lp + blockIdx.x] = t;
}

// z[0] = r[0] rounded through T (the value an FP32 preconditioner would pass on)
template <typename TZ, typename T>
__global__ void k_set_pinned_to(TZ *z, const TZ *r) {
  if (threadIdx.x == 0 && blockIdx.x == 0) z[0] = (TZ)(T)r[0];
}

template <typename T>
__global__ void k_negate(T *y, const T *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = -x[i];
}

// ---------------------------------------------------------------- precision helpers
template <typename T> struct Pr;
template <> struct Pr<double> {
  static const double *val(const Csr &A) { return A.val.p; }
  static double *w(MgLevel &L, int i) { return L.w64[i].p; }
  static DevBuf<double> &wb(MgLevel &L, int i) { return L.w64[i]; }
  static const double *dinv(const MgLevel &L) { return L.dinv.p; }
  static const double *cinv(const Mg &m) { return m.cinv.p; }
  static DevBuf<double> &inner(Ctx &c, int i) { return c.inner.v64[i]; }
};
template <> struct Pr<float> {
  static const float *val(const Csr &A) { return A.val32.p; }
  static float *w(MgLevel &L, int i) { return L.w32[i].p; }
  static DevBuf<float> &wb(MgLevel &L, int i) { return L.w32[i]; }
  static const float *dinv(const MgLevel &L) { return L.dinv32.p; }
  static const float *cinv(const Mg &m) { return m.cinv32.p; }
  static DevBuf<float> &inner(Ctx &c, int i) { return c.inner.v32[i]; }
};

static void ensure_fp32_mg(Ctx &c) {
  for (Mg *mg : {&c.mgu, &c.mgp})
    for (auto &L : mg->lv) {
      if (!L.A.val32.p) make_shadow(L.A, c.stream);
      if (L.P.nnz && !L.P.val32.p) make_shadow(L.P, c.stream);
      if (L.R.nnz && !L.R.val32.p) make_shadow(L.R, c.stream);
      if (!L.dinv32.p) {
        L.dinv32.alloc(L.dinv.n);
        convert(L.dinv32.p, L.dinv.p, (int64_t)L.dinv.n, c.stream);
      }
      for (int i = 0; i < 5; ++i)
        if (!L.w32[i].p) L.w32[i].alloc(L.w64[i].n);
    }
  if (!c.Mp.val32.p) make_shadow(c.Mp, c.stream);
}

// ---------------------------------------------------------------- Chebyshev smoothing
// `steps` Chebyshev iterations for A x = b preconditioned by D^{-1}, on the spectral
// interval [lmin, lmax] of D^{-1} A.  zero_init: start from x = 0.  x and x2 are
// ping-pong buffers; returns the buffer holding the result.  W = 4: 2x2 blocks (NC = 2).
template <typename T, int W, int NC>
static T *chebyshev(int64_t nrows, const int *rp, const int *col, const T *val, const T *dinv,
                    double lmin, double lmax, int steps, const T *b, T *x, T *x2, T *d,
                    bool zero_init, hipStream_t s, Prof *prof = nullptr) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  int k;
  if (zero_init) {
    hipLaunchKernelGGL((k_dinv_first<T, W, NC>), dim3(grid_for(nrows, 256)), dim3(256), 0, s, nrows,
                       dinv, b, (T)(1.0 / theta), d, x);
    FSI_CHECK_LAUNCH();
  } else {
    if (prof) prof->begin(s);
    spmv<T, W, NC, SP_CHEB>(nrows, rp, col, val, x, nrows, x2, nrows, s, b, d, dinv, (T)0,
                            (T)(1.0 / theta));
    if (prof) prof->end(s);
    std::swap(x, x2);
  }
  for (k = 1; k < steps; ++k) {
    double rho1 = 1.0 / (2.0 * sigma - rho);
    if (prof) prof->begin(s);
    spmv<T, W, NC, SP_CHEB>(nrows, rp, col, val, x, nrows, x2, nrows, s, b, d, dinv,
                            (T)(rho1 * rho), (T)(2.0 * rho1 / delta));
    if (prof) prof->end(s);
    std::swap(x, x2);
    rho = rho1;
  }
  return x;
}

// The same Chebyshev iteration with matrix-free products: first(scale, d, x) does the
// step from zero (d = x = scale D^{-1} b), step(x, x2, c1, c2) one step from x into x2.
// The same iteration on the velocity levels of the Q2 pair with the class stencils
// (q2_stencil) in place of the assembled rows; the first step from zero as chebyshev's.
template <typename T>
static T *chebyshev_q2(const MgLevel &L, const Q2Table<T> *tab, const T *dinv, double lmin, double lmax, int steps,
                       const T *b, T *x, T *x2, T *d, bool zero_init, hipStream_t s, Prof *prof = nullptr) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (zero_init) {
    hipLaunchKernelGGL((k_dinv_first<T, 4, 2>), dim3(grid_for(L.nodes, 256)), dim3(256), 0, s, L.nodes, dinv, b,
                       (T)(1.0 / theta), d, x);
    FSI_CHECK_LAUNCH();
  } else {
    if (prof) prof->begin(s);
    q2_stencil<T>(L.n, tab, x, b, d, x2, (T)0, (T)(1.0 / theta), false, s);
    if (prof) prof->end(s);
    std::swap(x, x2);
  }
  for (int k = 1; k < steps; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    if (prof) prof->begin(s);
    q2_stencil<T>(L.n, tab, x, b, d, x2, (T)(rho1 * rho), (T)(2.0 * rho1 / delta), false, s);
    if (prof) prof->end(s);
    std::swap(x, x2);
    rho = rho1;
  }
  return x;
}

template <typename T, typename First, typename Step>
static T *chebyshev_mf(First first, Step step, double lmin, double lmax, int steps, T *x, T *x2,
                       bool zero_init, hipStream_t s, Prof *prof) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (zero_init) {
    first((T)(1.0 / theta), x);
  } else {
    if (prof) prof->begin(s);
    step(x, x2, (T)0, (T)(1.0 / theta));
    if (prof) prof->end(s);
    std::swap(x, x2);
  }
  for (int k = 1; k < steps; ++k) {
    double rho1 = 1.0 / (2.0 * sigma - rho);
    if (prof) prof->begin(s);
    step(x, x2, (T)(rho1 * rho), (T)(2.0 * rho1 / delta));
    if (prof) prof->end(s);
    std::swap(x, x2);
    rho = rho1;
  }
  return x;
}

// Chebyshev on A_f (stencil) with right-hand side b and direction buffer d: the first three
// steps from zero (pre-smoothing) or the first three (else two) from x (post-smoothing) as
// one temporally blocked launch, further steps one launch each (same recurrence as
// chebyshev_mf; the profile brackets the post-smoothing launches, the largest single
// kernel of a step).
// out (optional, not zero_init): the last launch writes the result there instead of into a
// ping-pong buffer (returned); used to write a V-cycle's result into the caller's vector.
// out64 (optional, FP32 arithmetic, three steps from x): the result goes to that FP64 vector
// and the function returns nullptr.
// xc (optional, at least three steps from x): the steps start from x + P xc, the coarse
// correction of lattice n / 2 (lane stride lc) added by the fused launch.
template <typename T>
static T *chebyshev_stencil(int n, const StencilTable<T> *tab, double lmin, double lmax, int steps,
                            const T *b, T *x, T *x2, T *d, bool zero_init, hipStream_t s, Prof *prof,
                            int K = 1, int64_t ls = 0, T *out = nullptr, double *out64 = nullptr,
                            const T *xc = nullptr, int64_t lc = 0, LP<double> dot = LP<double>(),
                            LP<const double> b64 = LP<const double>()) {
  FSI_REQUIRE(!xc || (!zero_init && steps >= 3), FSI_E_STATE, "the coarse correction rides on the fused steps");
  FSI_REQUIRE(!dot.p || (!zero_init && steps == 3), FSI_E_STATE, "the tile sums ride on the last fused launch");
  const LP<const T> lxc(xc, lc);
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  auto next = [&](T &c1, T &c2) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    c1 = (T)(rho1 * rho);
    c2 = (T)(2.0 * rho1 / delta);
    rho = rho1;
  };
  const LP<const T> lb(b, ls);
  const LP<T> ld(d, ls);
  // the fused launches store their last direction only for the single steps that follow
  const LP<T> ld3 = steps > 3 ? ld : LP<T>();
  int done = 0;
  if (zero_init && steps >= 3) {
    T c1a, c2a, c1b, c2b;
    next(c1a, c2a);
    next(c1b, c2b);
    cheb2_pre<T>(n, tab, lb, ld3, LP<T>(x, ls), (T)(1.0 / theta), c1a, c2a, c1b, c2b, s, K);
    done = 3;
  } else if (!zero_init && steps == 3 && out64) {
    T c1b, c2b, c1c, c2c;
    next(c1b, c2b);
    next(c1c, c2c);
    if (prof) prof->begin(s);
    cheb3_post<T, double>(n, tab, LP<const T>(x, ls), lb, LP<T>(), LP<double>(out64, ls), (T)(1.0 / theta), c1b, c2b,
                          c1c, c2c, s, K, lxc, dot, b64);
    if (prof) prof->end(s);
    return nullptr;
  } else if (!zero_init && steps >= 3) {
    T c1b, c2b, c1c, c2c;
    next(c1b, c2b);
    next(c1c, c2c);
    T *dst = (out && steps == 3) ? out : x2;
    if (prof) prof->begin(s);
    cheb3_post<T>(n, tab, LP<const T>(x, ls), lb, ld3, LP<T>(dst, ls), (T)(1.0 / theta), c1b, c2b, c1c, c2c, s, K,
                  lxc, dot, b64);
    if (prof) prof->end(s);
    x2 = x;
    x = dst;
    done = 3;
  } else if (!zero_init && steps >= 2) {
    T c1b, c2b;
    next(c1b, c2b);
    T *dst = (out && steps == 2) ? out : x2;
    if (prof) prof->begin(s);
    cheb2_post<T>(n, tab, LP<const T>(x, ls), lb, steps > 2 ? ld : LP<T>(), LP<T>(dst, ls), (T)(1.0 / theta), c1b,
                  c2b, s, K);
    if (prof) prof->end(s);
    x2 = x;
    x = dst;
    done = 2;
  } else if (zero_init) {
    p2_first<T>(n, tab, lb, (T)(1.0 / theta), ld, LP<T>(x, ls), s, K);
    done = 1;
  } else {
    T *dst = (out && steps == 1) ? out : x2;
    stencil_launch<T, SP_CHEB>(n, tab, LP<const T>(x, ls), lb, ld, LP<T>(dst, ls), (T)0, (T)(1.0 / theta), s, K);
    x2 = x;
    x = dst;
    done = 1;
  }
  for (int k = done; k < steps; ++k) {
    T c1, c2;
    next(c1, c2);
    T *dst = (out && k == steps - 1) ? out : x2;
    stencil_launch<T, SP_CHEB>(n, tab, LP<const T>(x, ls), lb, ld, LP<T>(dst, ls), c1, c2, s, K);
    x2 = x;
    x = dst;
  }
  return x;
}

template <typename T>
static T *chebyshev_p1(int n, const P1Table<T> *tab, double lmin, double lmax, int steps, const T *b,
                       T *x, T *x2, T *d, bool zero_init, hipStream_t s, int K = 1, int64_t ls = 0) {
  const LP<const T> lb(b, ls);
  const LP<T> ld(d, ls);
  return chebyshev_mf<T>([&](T sc, T *xo) { p1_first<T>(n, tab, lb, sc, ld, LP<T>(xo, ls), s, K); },
                         [&](const T *xi, T *xo, T c1, T c2) {
                           p1_launch<T, SP_CHEB>(n, tab, LP<const T>(xi, ls), lb, ld, LP<T>(xo, ls), c1, c2, s,
                                                 K);
                         },
                         lmin, lmax, steps, x, x2, zero_init, s, nullptr);
}

// The Chebyshev coefficients of chebyshev_mf: step k updates d = c1[k] d + c2[k] D^{-1} r
// (from zero, step 0 is x = d = c2[0] D^{-1} b; from x, c1[0] = 0).
template <typename T>
static void p1_cheb_coefs(double lmin, double lmax, int steps, T *c1, T *c2) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  c1[0] = (T)0;
  c2[0] = (T)(1.0 / theta);
  for (int k = 1; k < steps; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    c1[k] = (T)(rho1 * rho);
    c2[k] = (T)(2.0 * rho1 / delta);
    rho = rho1;
  }
}

// The steps of chebyshev_p1 (2 or 3, the same coefficients) in one launch (k_p1_multi): the
// result goes to y.  Returns false for other step counts.
template <typename T>
static bool p1_cheb_fused(int n, const P1Table<T> *tab, double lmin, double lmax, int steps, const T *b, const T *x,
                          T *y, bool zero, hipStream_t s, int K, int64_t ls) {
  if (steps != 2 && steps != 3) return false;
  P1MultiArgs<T, T> a{};
  a.n = n;
  a.tab = tab;
  a.b = b;
  a.x = x;
  a.y = y;
  a.lb = ls;
  p1_cheb_coefs<T>(lmin, lmax, steps, a.c1, a.c2);
  if (steps == 2) {
    if (zero) p1_multi<T, T, 2, true, P1_OUT_X>(a, s, K);
    else p1_multi<T, T, 2, false, P1_OUT_X>(a, s, K);
  } else {
    if (zero) p1_multi<T, T, 3, true, P1_OUT_X>(a, s, K);
    else p1_multi<T, T, 3, false, P1_OUT_X>(a, s, K);
  }
  return true;
}

template <typename T> static const StencilTable<T> *stab(const MgLevel &L);
template <> const StencilTable<double> *stab<double>(const MgLevel &L) {
  return (const StencilTable<double> *)L.stab64.p;
}
template <> const StencilTable<float> *stab<float>(const MgLevel &L) {
  return (const StencilTable<float> *)L.stab32.p;
}
template <typename T> static const P1Table<T> *p1tab(const MgLevel &L) {
  return (const P1Table<T> *)(std::is_same<T, double>::value ? L.p1tab64.p : L.p1tab32.p);
}
template <typename T> static const P2RestrTable<T> *rtab(const Mg &mg) {
  return (const P2RestrTable<T> *)(std::is_same<T, double>::value ? mg.rtab64.p : mg.rtab32.p);
}

// The arguments of the one-launch coarse end of the velocity V-cycle from level l (l >= 1,
// where the restricted right-hand side vanishes at Dirichlet nodes), or false when the
// remaining levels do not fit it (too fine, too many, smoothing degree or LDS).
template <typename T>
static bool tail_args(Mg &mg, int l, int degree, const T *b, T *x, int64_t ls, TailArgs<T> &a) {
  const int last = (int)mg.lv.size() - 1;   // the dense coarsest level
  const int nlev = last - l;
  if (!mg.stencil || mg.comps != 2 || l < 1 || nlev < 1 || nlev > kTailMax || degree < 1 || degree > kTailDeg ||
      mg.lv[l].n > kTailMaxN)
    return false;
  a = TailArgs<T>{};
  a.nlev = nlev;
  a.degree = degree;
  int off = 0;
  for (int k = 0; k < nlev; ++k) {
    const MgLevel &L = mg.lv[l + k];
    TailLevel<T> &t = a.lv[k];
    t.n = L.n;
    t.off = off;
    off += 4 * tail_plane_entries(L.n);
    t.tab = stab<T>(L);
    // the coefficients of chebyshev_stencil on [lmax / 15, lmax]
    const double lmax = L.lmax, lmin = L.lmax / 15.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    t.s = (T)(1.0 / theta);
    for (int j = 0; j + 1 < degree; ++j) {
      const double rho1 = 1.0 / (2.0 * sigma - rho);
      t.c1[j] = (T)(rho1 * rho);
      t.c2[j] = (T)(2.0 * rho1 / delta);
      rho = rho1;
    }
  }
  a.offd = off;
  off += 2 * tail_plane_entries(mg.lv[l].n);
  a.offc = off;
  a.m = (int)mg.ncoarse;
  FSI_REQUIRE(a.m == 2 * (int)mg.lv[last].nodes, FSI_E_STATE, "coarsest level size");
  if (a.m > kTailDenseMax) return false;
  off += 2 * a.m;
  a.offt = off;
  off += nlev * kTailTab + kTailRw;
  a.lds = off;
  if ((int64_t)a.lds * (int64_t)sizeof(T) > tail_lds_limit()) return false;
  // the dense inverse in LDS too when it fits (loaded with the tables at the start)
  a.offm = -1;
  if ((int64_t)(off + (int64_t)a.m * a.m) * (int64_t)sizeof(T) <= tail_lds_limit()) {
    a.offm = off;
    a.lds = off + a.m * a.m;
  }
  a.rt = rtab<T>(mg);
  a.cinv = Pr<T>::cinv(mg);
  a.b = b;
  a.x = x;
  a.lb = ls;
  return true;
}

// The arguments of the one-launch coarse end of the pressure V-cycle from level l, or false
// when the remaining levels do not fit it (too fine, too many, smoothing degree or LDS).
template <typename T>
static bool p1_tail_args(Mg &mg, int l, int degree, const T *b, T *x, int64_t ls, PTailArgs<T> &a) {
  const int last = (int)mg.lv.size() - 1;   // the dense coarsest level
  const int nlev = last - l;
  if (!mg.stencil || mg.comps != 1 || nlev < 1 || nlev > kPTailMax || degree < 1 || degree > kPTailDeg ||
      mg.lv[l].n > kPTailMaxN || (mg.lv[l].n + 1) * (mg.lv[l].n + 1) > kPTailPer * 1024)
    return false;
  a = PTailArgs<T>{};
  a.nlev = nlev;
  a.degree = degree;
  int off = 0;
  for (int k = 0; k < nlev; ++k) {
    const MgLevel &L = mg.lv[l + k];
    PTailLevel<T> &t = a.lv[k];
    t.n = L.n;
    t.off = off;
    off += 2 * (L.n + 1) * (L.n + 1);
    t.tab = p1tab<T>(L);
    // the coefficients of the per-level launches on [lmax / 30, lmax]
    p1_cheb_coefs<T>(L.lmax / 30.0, L.lmax, degree, t.c1, t.c2);
  }
  a.offx2 = off;
  off += (mg.lv[l].n + 1) * (mg.lv[l].n + 1);
  a.offc = off;
  a.m = (int)mg.ncoarse;
  FSI_REQUIRE(a.m == (int)mg.lv[last].nodes, FSI_E_STATE, "coarsest level size");
  if (a.m > kPTailDenseMax) return false;
  off += 2 * a.m;
  a.offt = off;
  off += nlev * kPTailTab;
  a.lds = off;
  if ((int64_t)a.lds * (int64_t)sizeof(T) > tail_lds_limit()) return false;
  a.offm = -1;
  if ((int64_t)(off + (int64_t)a.m * a.m) * (int64_t)sizeof(T) <= tail_lds_limit()) {
    a.offm = off;
    a.lds = off + a.m * a.m;
  }
  a.cinv = Pr<T>::cinv(mg);
  a.b = b;
  a.x = x;
  a.lb = ls;
  return true;
}

// ---------------------------------------------------------------- V-cycle
// One V-cycle at level l for right-hand side b (comps * nodes entries, component-major).
// Returns the level work vector that holds the result.
// out (optional): where the matrix-free velocity cycle writes its result (the returned
// pointer); otherwise a level work vector.  out64 (optional, FP32 cycle): an FP64 vector the
// result goes to when the last smoothing launch can store it there (then nullptr is returned).
// dot (optional, level 0 of a velocity cycle with tile_dot_ok): the last launch stores the
// per-tile sums of b . result (cheb3_dot_count(n) per lane), with b64 (FP32 cycle) in place
// of b.
template <typename T, int W, int NC>
static T *vcycle(Mg &mg, int l, const T *b, hipStream_t s, Prof *prof = nullptr, int K = 1, T *out = nullptr,
                 double *out64 = nullptr, LP<double> dot = LP<double>(),
                 LP<const double> b64 = LP<const double>()) {
  MgLevel &L = mg.lv[l];
  T *x = Pr<T>::w(L, 0), *x2 = Pr<T>::w(L, 4), *r = Pr<T>::w(L, 2), *d = Pr<T>::w(L, 3);
  // K systems (matrix-free hierarchy only): lane k of every level vector at + k comps nodes
  FSI_REQUIRE(K == 1 || mg.stencil, FSI_E_STATE, "several systems per V-cycle need the matrix-free smoother");
  FSI_REQUIRE(!dot.p || (l == 0 && W == 4 && mg.stencil && l + 1 < (int)mg.lv.size()), FSI_E_STATE,
              "tile sums only from the finest velocity level of a matrix-free cycle");
  const int64_t ls = (int64_t)mg.comps * L.nodes;
  if (l + 1 == (int)mg.lv.size()) {
    dense_mv<T>((int)mg.ncoarse, Pr<T>::cinv(mg), b, x, K, s);
    return x;
  }
  // Chebyshev interval [lmax / R, lmax] of D^{-1} A: R = 15 on the velocity levels, 30 on the
  // pressure levels (measured at 1024^2: R = 30 / 15 / 10 / 5 on the velocity levels gave 228 /
  // 174 / 204 / 228 inner steps per FP64 step; the pressure levels are best left at 30)
  const double lmax = L.lmax, lmin = L.lmax / (W == 4 ? 15.0 : 30.0);
  const int degree = std::is_same<T, float>::value ? mg.degree32 : mg.degree;
  const T *dinv = Pr<T>::dinv(L);
  const T *val = Pr<T>::val(L.A);
  Prof *pl = (l == 0) ? prof : nullptr;
  MgLevel &C = mg.lv[l + 1];
  T *bc = Pr<T>::w(C, 1);
  const int64_t lc = (int64_t)mg.comps * C.nodes;
  if constexpr (W == 4) {   // the coarse end of the velocity cycle in one launch
    TailArgs<T> ta;
    if (mg.tail && tail_args<T>(mg, l, degree, b, x, ls, ta)) {
      mg_tail<T>(ta, s, K);
      return x;
    }
  } else {                  // the coarse end of the pressure cycle in one launch
    PTailArgs<T> pa;
    if (mg.tail && p1_tail_args<T>(mg, l, degree, b, x, ls, pa)) {
      p1_tail<T>(pa, s, K);
      return x;
    }
  }
  if (mg.stencil) {   // matrix-free smoothing, residual and transfers
    // velocity levels with three or more post-smoothing steps: the fused launch adds the
    // coarse correction while it stages x (no separate prolongation pass)
    const bool fuse = W == 4 && degree >= 3;
    auto smooth = [&](T *x0, T *x1, bool zero, const T *xcor) -> T * {
      if constexpr (W == 4)
        return chebyshev_stencil<T>(L.n, stab<T>(L), lmin, lmax, degree, b, x0, x1, d, zero, s, pl, K, ls,
                                    zero ? nullptr : out, zero ? nullptr : out64, xcor, lc,
                                    zero ? LP<double>() : dot, zero ? LP<const double>() : b64);
      else if (p1_cheb_fused<T>(L.n, p1tab<T>(L), lmin, lmax, degree, b, x0, zero ? x0 : x1, zero, s, K, ls))
        return (void)xcor, zero ? x0 : x1;
      else
        return (void)xcor, chebyshev_p1<T>(L.n, p1tab<T>(L), lmin, lmax, degree, b, x0, x1, d, zero, s, K, ls);
    };
    T *xs = smooth(x, x2, true, nullptr);
    T *xo = (xs == x) ? x2 : x;
    if constexpr (W == 4) {   // the fine residual stays in LDS
      (void)r;
      resid_restrict<T>(L.n, stab<T>(L), rtab<T>(mg), LP<const T>(xs, ls), LP<const T>(b, ls), LP<T>(bc, lc), s, K);
    } else {
      p1_launch<T, SP_RESID>(L.n, p1tab<T>(L), LP<const T>(xs, ls), LP<const T>(b, ls), LP<T>(), LP<T>(r, ls),
                             (T)0, (T)0, s, K);
      p1_restrict<T>(L.n, LP<const T>(r, ls), LP<T>(bc, lc), s, K);
    }
    T *xc = vcycle<T, W, NC>(mg, l + 1, bc, s, nullptr, K);
    if constexpr (W == 4) {
      if (!fuse) p2_prolong_add<T>(L.n, LP<const T>(xc, lc), LP<T>(xs, ls), s, K);
    } else {
      p1_prolong_add<T>(L.n, LP<const T>(xc, lc), LP<T>(xs, ls), s, K);
    }
    return smooth(xs, xo, false, fuse ? xc : nullptr);
  }
  // the Q2 pair's velocity levels: class stencils for the smoothing steps and the residual
  const Q2Table<T> *q2 = nullptr;
  if constexpr (W == 4)
    q2 = (const Q2Table<T> *)(std::is_same<T, double>::value ? L.q2tab64.p : L.q2tab32.p);
  T *xs = q2 ? chebyshev_q2<T>(L, q2, dinv, lmin, lmax, degree, b, x, x2, d, true, s, pl)
             : chebyshev<T, W, NC>(L.A.nrows, L.A.rowptr.p, L.A.col.p, val, dinv, lmin, lmax, degree, b, x,
                                   x2, d, true, s, pl);
  T *xo = (xs == x) ? x2 : x;
  if (q2) q2_stencil<T>(L.n, q2, xs, b, nullptr, r, (T)0, (T)0, true, s);
  else spmv<T, W, NC, SP_RESID>(L.A.nrows, L.A.rowptr.p, L.A.col.p, val, xs, L.nodes, r, L.nodes, s, b);
  spmv<T, 1, NC, SP_APPLY>(L.R.nrows, L.R.rowptr.p, L.R.col.p, Pr<T>::val(L.R), r, L.nodes, bc,
                           C.nodes, s);
  T *xc = vcycle<T, W, NC>(mg, l + 1, bc, s);
  spmv<T, 1, NC, SP_ADD>(L.P.nrows, L.P.rowptr.p, L.P.col.p, Pr<T>::val(L.P), xc, C.nodes, xs,
                         L.nodes, s);
  if (q2) return chebyshev_q2<T>(L, q2, dinv, lmin, lmax, degree, b, xs, xo, d, false, s, pl);
  return chebyshev<T, W, NC>(L.A.nrows, L.A.rowptr.p, L.A.col.p, val, dinv, lmin, lmax, degree, b,
                             xs, xo, d, false, s, pl);
}

// ---------------------------------------------------------------- A11 preconditioner
template <typename T> static const T *mp_dinv(Ctx &c);
template <> const double *mp_dinv<double>(Ctx &c) { return c.Mp_dinv.p; }
template <> const float *mp_dinv<float>(Ctx &c) { return c.Mp_dinv32.p; }

// Chebyshev-Jacobi steps of the pressure mass inverse inside the Schur approximation
// (measured with the final multigrid, inner steps per step at 1024^2 / 256^2 / 512^2:
// 4 steps 163/201/81, 3 steps 144/204/83, 2 steps 229/228/92; 3 is the fastest overall)
constexpr int kMpSteps = 3;

// z = diag(V, S^{-1}) r on [u | p], for K systems at once (lane k of r and z at + k nf,
// nf = 2 N2 + Np; K > 1 needs the matrix-free hierarchies).  The two blocks share no
// buffer: outside graph capture the pressure part runs on the auxiliary stream beside the
// velocity V-cycle (both chains are latency-bound on the coarse levels), forked after the
// producer of r and joined before the consumer of z.  Captured graphs keep the whole
// preconditioner on one stream.
// r64, z64 (FP32 arithmetic, one system): the results are stored straight into the FP64 vector
// z64 (z unused) and the pressure residual is read from r64 (r holds the velocity part).
// dot (FP64 form, tile_dot_ok): the launches that write z also store per-tile / per-block
// parts of r . z: cheb3_dot_count(n) velocity tile sums, then kPresDotBlocks pressure
// block sums, per lane (lane stride dot.s).
// part: PC_BOTH, or only the velocity cycle (PC_VEL) or only the pressure part (PC_PRES); the
// other part of z is left as it is.
enum { PC_BOTH = 0, PC_VEL = 1, PC_PRES = 2 };
template <typename T>
static void a11_precond(Ctx &c, const T *r, T *z, int K = 1, const double *r64 = nullptr, double *z64 = nullptr,
                        LP<double> dot = LP<double>(), int part = PC_BOTH) {
  FSI_REQUIRE((!dot.p || std::is_same<T, double>::value || r64), FSI_E_STATE,
              "sums of r . z in the FP32 form need the FP64 residual");
  FSI_REQUIRE(!dot.p || part == PC_BOTH, FSI_E_STATE, "the sums of r . z need both parts");
  const bool fork = !c.capturing && part == PC_BOTH;
  hipStream_t s = c.stream, sp = fork ? c.aux_stream : c.stream;
  const int64_t N2 = c.N2, Np = c.Np, nf = 2 * N2 + Np;
  Prof *pf = std::is_same<T, double>::value ? &c.prof64 : &c.prof32;
  if (fork) {
    FSI_HIP(hipEventRecord(c.ev_fork, s));
    FSI_HIP(hipStreamWaitEvent(sp, c.ev_fork, 0));
  }
  if (part == PC_PRES) {
    // the velocity cycle is not run
  } else if (z64) {
    T *xu = vcycle<T, 4, 2>(c.mgu, 0, r, s, pf->on ? pf : nullptr, 1, nullptr, z64, dot,
                            LP<const double>(dot.p ? r64 : nullptr));
    FSI_REQUIRE(!dot.p || !xu, FSI_E_STATE, "the sums of r . z need the direct FP64 output");
    if (xu) convert(z64, xu, 2 * N2, s);
  } else if (K == 1) {   // the cycle reads r and writes z in place (one system: no lane stride)
    T *xu = vcycle<T, 4, 2>(c.mgu, 0, r, s, pf->on ? pf : nullptr, 1, z, nullptr, dot);
    if (xu != z) convert(z, xu, 2 * N2, s);
  } else {   // the finest level's right-hand side: the velocity part of each lane, contiguous
    T *bu = Pr<T>::w(c.mgu.lv[0], 1);
    convert_l(LP<T>(bu, 2 * N2), LP<const T>(r, nf), 2 * N2, s, K);
    T *xu = vcycle<T, 4, 2>(c.mgu, 0, bu, s, nullptr, K, nullptr, nullptr, dot,
                            LP<const double>(dot.p && r64 ? r64 : nullptr, nf));
    convert_l(LP<T>(z, nf), LP<const T>(xu, 2 * N2), 2 * N2, s, K);
  }
  if (part == PC_VEL) {
    FSI_CHECK_LAUNCH();
    return;
  }
  // r' = pressure residual with the pinned entry removed (keeps the operator symmetric)
  T *rp = Pr<T>::inner(c, 8).p;
  if (z64) convert(rp, r64 + 2 * N2, Np, sp);
  else convert_l(LP<T>(rp, Np), LP<const T>(r + 2 * N2, nf), Np, sp, K);
  fill_l(LP<T>(rp, Np), 1, (T)0, sp, K);
  T *xp = vcycle<T, 1, 1>(c.mgp, 0, rp, sp, nullptr, K);
  if (c.pair == FSI_PAIR_Q2P1DISC) {   // M_p of the discontinuous pressure is diagonal: no mass solve
    FSI_REQUIRE(!dot.p && K == 1, FSI_E_STATE, "the Q2 / P1-disc pair runs one system and forms no tile sums");
    if (z64)
      hipLaunchKernelGGL((k_q_pres<double, T>), dim3(vgrid(Np)), dim3(256), 0, sp, z64 + 2 * N2, r64 + 2 * N2, xp,
                         mp_dinv<T>(c), (T)c.nu, (T)(c.rho / c.dt), Np);
    else
      hipLaunchKernelGGL((k_q_pres<T, T>), dim3(vgrid(Np)), dim3(256), 0, sp, z + 2 * N2, r + 2 * N2, xp,
                         mp_dinv<T>(c), (T)c.nu, (T)(c.rho / c.dt), Np);
    FSI_CHECK_LAUNCH();
    if (fork) {
      FSI_HIP(hipEventRecord(c.ev_join, sp));
      FSI_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
    }
    return;
  }
  if (c.mgp.stencil) {
    // the mass solve (kMpSteps Chebyshev steps from zero) and the output z_p = nu x + (rho/dt) x_L
    // with the pinned entry and the parts of r . z, in one launch
    static_assert(kMpSteps == 3, "the fused mass solve takes three steps");
    const P1Table<T> *mtab = (const P1Table<T> *)(std::is_same<T, double>::value ? c.mptab64.p : c.mptab32.p);
    double *part = dot.p ? dot.p + cheb3_dot_count(c.n) : nullptr;
    if (z64) {
      P1MultiArgs<T, double> a{};
      a.n = c.n;
      a.tab = mtab;
      a.b = rp;
      p1_cheb_coefs<T>(0.5, 2.0, kMpSteps, a.c1, a.c2);
      a.z = z64 + 2 * N2;
      a.r = r64 + 2 * N2;
      a.w = xp;
      a.a = (T)c.nu;
      a.b2 = (T)(c.rho / c.dt);
      a.part = part;
      a.lb = Np;
      a.lz = nf;
      a.lp = dot.s;
      p1_multi<T, double, 3, true, P1_OUT_SCHUR>(a, sp, 1);
    } else {
      P1MultiArgs<T, T> a{};
      a.n = c.n;
      a.tab = mtab;
      a.b = rp;
      p1_cheb_coefs<T>(0.5, 2.0, kMpSteps, a.c1, a.c2);
      a.z = z + 2 * N2;
      a.r = r + 2 * N2;
      a.r64 = r64 ? r64 + 2 * N2 : nullptr;
      a.w = xp;
      a.a = (T)c.nu;
      a.b2 = (T)(c.rho / c.dt);
      a.part = part;
      a.lb = Np;
      a.lz = nf;
      a.lp = dot.s;
      p1_multi<T, T, 3, true, P1_OUT_SCHUR>(a, sp, K);
    }
    FSI_CHECK_LAUNCH();
    if (fork) {
      FSI_HIP(hipEventRecord(c.ev_join, sp));
      FSI_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
    }
    return;
  }
  // mass solve scratch: x, x2, d of every lane (3 Np each) in one inner vector
  T *mx = Pr<T>::inner(c, 7).p, *mx2 = mx + (int64_t)K * Np, *md = mx + 2 * (int64_t)K * Np;
  T *mres = c.mgp.stencil
                ? chebyshev_p1<T>(c.n, (const P1Table<T> *)(std::is_same<T, double>::value ? c.mptab64.p
                                                                                          : c.mptab32.p),
                                  0.5, 2.0, kMpSteps, rp, mx, mx2, md, true, sp, K, Np)
                : chebyshev<T, 1, 1>(Np, c.Mp.rowptr.p, c.Mp.col.p, Pr<T>::val(c.Mp), mp_dinv<T>(c), 0.5,
                                     2.0, kMpSteps, rp, mx, mx2, md, true, sp);
  if (z64 && dot.p) {
    hipLaunchKernelGGL((k_pres_out_dot<double, T>), dim3(kPresDotBlocks, 1), dim3(kRedBlock), 0, sp, z64 + 2 * N2,
                       r64 + 2 * N2, mres, xp, (T)c.nu, (T)(c.rho / c.dt), Np, nf, Np,
                       dot.p + cheb3_dot_count(c.n), dot.s, nullptr);
  } else if (z64) {
    lincomb_to<double, T>(z64 + 2 * N2, mres, xp, (T)c.nu, (T)(c.rho / c.dt), Np, sp);
    hipLaunchKernelGGL((k_set_pinned_to<double, T>), dim3(1), dim3(1), 0, sp, z64 + 2 * N2, r64 + 2 * N2);
  } else if (dot.p) {
    hipLaunchKernelGGL((k_pres_out_dot<T, T>), dim3(kPresDotBlocks, K), dim3(kRedBlock), 0, sp, z + 2 * N2,
                       r + 2 * N2, mres, xp, (T)c.nu, (T)(c.rho / c.dt), Np, nf, Np,
                       dot.p + cheb3_dot_count(c.n), dot.s, r64 ? r64 + 2 * N2 : nullptr);
  } else {
    lincomb_l(LP<T>(z + 2 * N2, nf), LP<const T>(mres, Np), LP<const T>(xp, Np), (T)c.nu, (T)(c.rho / c.dt), Np,
              sp, K);
    hipLaunchKernelGGL(k_set_pinned<T>, dim3(1, K), dim3(1), 0, sp, z + 2 * N2, r + 2 * N2, nf);
  }
  FSI_CHECK_LAUNCH();
  if (fork) {
    FSI_HIP(hipEventRecord(c.ev_join, sp));
    FSI_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
  }
}

// ---------------------------------------------------------------- inner MINRES
// The A11 preconditioner on FP64 vectors with arithmetic TA: FP32 runs on a converted copy
// of the velocity residual (read three times by the finest level) and stores its results
// straight into z; several systems run on converted copies of whole vectors.
template <typename TA>
static void a11_precond_on64(Ctx &c, const double *r, double *z, int K = 1, int part = PC_BOTH) {
  if constexpr (std::is_same<TA, double>::value) {
    a11_precond<double>(c, r, z, K, nullptr, nullptr, LP<double>(), part);
  } else if (K == 1) {
    if (part != PC_PRES) convert(c.outer.x32.p, r, 2 * c.N2, c.stream);
    a11_precond<float>(c, c.outer.x32.p, nullptr, 1, r, z, LP<double>(), part);
  } else {
    const int64_t nf = 2 * c.N2 + c.Np, nv = 2 * c.N2;
    convert_l(LP<float>(c.outer.x32.p, nf), LP<const double>(r, nf), nf, c.stream, K);
    a11_precond<float>(c, c.outer.x32.p, c.outer.y32.p, K, nullptr, nullptr, LP<double>(), part);
    if (part != PC_PRES)
      convert_l(LP<double>(z, nf), LP<const float>(c.outer.y32.p, nf), nv, c.stream, K);
    if (part != PC_VEL)
      convert_l(LP<double>(z + nv, nf), LP<const float>(c.outer.y32.p + nv, nf), nf - nv, c.stream, K);
  }
}

// Capture `body` (kernel launches on c.stream) into an executable graph; the capture runs
// on the context's capture stream (the NULL stream cannot be captured) and only records.
template <typename Body>
static void capture_graph(Ctx &c, hipGraphExec_t &ge, Body body) {
  hipStream_t s = c.stream;
  if (!c.cap_stream) FSI_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  FSI_HIP(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
  c.stream = c.cap_stream;
  c.capturing = true;
  try {
    body();
  } catch (...) {
    c.stream = s;
    c.capturing = false;
    (void)hipStreamEndCapture(c.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  c.stream = s;
  c.capturing = false;
  FSI_HIP(hipStreamEndCapture(c.cap_stream, &g));
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  FSI_HIP(e);
}

// The preconditioner through a HIP graph: captured once per precision and lane count on the
// staging buffers (a fixed sequence of kernels with fixed arguments), then replayed.  Only
// kernel nodes are captured (copies are kernels too).
template <typename TA>
static void a11_precond_graph(Ctx &c, const double *r, double *z, int K) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np;
  const int k = std::is_same<TA, double>::value ? 0 : 1;
  convert_l(LP<double>(c.pc_in.p, nf), LP<const double>(r, nf), nf, s, K);
  hipGraphExec_t &ge = c.pc_graph[k][K];
  if (!ge) capture_graph(c, ge, [&] { a11_precond_on64<TA>(c, c.pc_in.p, c.pc_out.p, K); });
  FSI_HIP(hipGraphLaunch(ge, s));
  convert_l(LP<double>(z, nf), LP<const double>(c.pc_out.p, nf), nf, s, K);
}

template <typename TA>
static void a11_precond_any(Ctx &c, const double *r, double *z, int K = 1) {
  const bool profiling = c.prof64.on || c.prof32.on;
  if (c.use_graphs && !profiling) a11_precond_graph<TA>(c, r, z, K);
  else a11_precond_on64<TA>(c, r, z, K);
}

void Ctx::drop_graphs() {
  for (auto &row : pc_graph)
    for (auto &g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  for (auto &per_k : ms_graph)
    for (auto &row : per_k)
      for (auto &g : row)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
}

// Preconditioned MINRES (Paige-Saunders recurrences) for A11 x = b from x = 0; stops when
// the preconditioned residual estimate falls below tol times its initial value.  The
// Lanczos vectors, dot products, updates and the A11 product are FP64 in every mode; TA is
// the arithmetic of the preconditioner (V-cycle, Chebyshev mass solve, pressure V-cycle).
// An FP32 product of A_f on a smooth vector loses about kappa * eps_32 (0.06 at 1024^2
// cells) to cancellation, which stalls the recurrence; inside the V-cycle the residuals
// are not smooth-dominated and FP32 arithmetic costs the preconditioner nothing.
//
// The scalar recurrence runs on the device (one thread), so an iteration is a fixed
// sequence of kernels: on small grids it is replayed as a captured graph (one per rotation
// of the Lanczos buffers) and the host looks at the convergence flag every few iterations.
//
// Directions and iterate in blocks.  The recurrence w_j = (v_j - e_j w_{j-2} - d_j w_{j-1})
// / gamma_j, x += phi_j w_j is not applied vector by vector each iteration (six vector passes
// per iteration).  Each iteration stores its Lanczos vector v_j in a slot of a block of up to
// ms_B vectors and records (e_j, d_j, 1/gamma_j, phi_j); after ms_B iterations, and at the
// end, the same recurrence is run on coefficient vectors over the basis (v slots, w_{k0-1},
// w_{k0}) and one pass forms x, w_{k-1} and w_k as those combinations (ms_B + 3 reads and 3
// writes per block).  Once converged, a lane records no more updates, so its x does not
// depend on how often the host checks, nor on the other lanes of a batch.
struct MinresState {
  double alfa, beta2;                         // dot products of the iteration
  double beta, oldb, dbar, epsln, phibar, cs, sn, beta1, tol;
  double s, c_r1;                             // 1 / beta, -beta / oldb
  double e, d, ginv, phi;                     // direction update
  double it, done, apply;                     // iterations; converged; update valid
  double slot;                                // slot of this iteration's Lanczos vector
};
constexpr int kMsRec = 5;                     // recorded per iteration: e, d, 1/gamma, phi, applied
constexpr int kMsBMax = 32;                   // Lanczos vectors per block at most
static_assert(kMsBMax + 2 <= kWave, "one wave computes the coefficients of a block");
constexpr int kMsDoubles = sizeof(MinresState) / sizeof(double);
constexpr int kMsLagMaxN = 256;   // grids whose inner steps read the state back one step late
constexpr int kHpinHalf = 2048;   // doubles: the two halves of the pinned host buffer

// The kernels below run K systems (lane = blockIdx.y): lane k uses st + k and vectors at
// + k n (n = nf, the lane stride of every inner vector).
__global__ void k_ms_init(MinresState *st, double tol) {
  if (threadIdx.x || blockIdx.x) return;
  st += blockIdx.y;
  double b2 = st->beta2;
  double b = (b2 > 0.0 && b2 == b2) ? sqrt(b2) : 0.0;
  st->beta = st->beta1 = st->phibar = b;
  st->oldb = st->dbar = st->epsln = st->sn = 0.0;
  st->cs = -1.0;
  st->tol = tol;
  st->s = b > 0.0 ? 1.0 / b : 0.0;
  st->c_r1 = 0.0;
  st->it = 0.0;
  st->done = b > 0.0 ? 0.0 : 1.0;
  st->apply = 0.0;
  st->slot = 0.0;
}

// After the two dot products of an iteration: Givens rotation and the next coefficients,
// recorded in slot st->slot of the lane's history (B slots of kMsRec; the host starts a new
// block before the slots run out, and a slot out of range records nothing).
__device__ void ms_step(MinresState *st, double *hist, int B) {
  const int sl = (int)st->slot;
  double *h = (sl >= 0 && sl < B) ? hist + kMsRec * sl : nullptr;
  st->slot += 1.0;
  if (st->done != 0.0) {
    st->apply = 0.0;
    if (h) h[4] = 0.0;
    return;
  }
  const double alfa = st->alfa, nb2 = st->beta2;
  const double oldb = st->beta;
  const double beta = sqrt(nb2 > 0.0 ? nb2 : 0.0);
  const double oldeps = st->epsln;
  const double delta = st->cs * st->dbar + st->sn * alfa;
  const double gbar = st->sn * st->dbar - st->cs * alfa;
  st->epsln = st->sn * beta;
  st->dbar = -st->cs * beta;
  double gamma = sqrt(gbar * gbar + beta * beta);
  if (gamma < 1e-300) gamma = 1e-300;
  st->cs = gbar / gamma;
  st->sn = beta / gamma;
  st->phi = st->cs * st->phibar;
  st->phibar = st->sn * st->phibar;
  st->e = oldeps;
  st->d = delta;
  st->ginv = 1.0 / gamma;
  st->apply = 1.0;
  if (h) {
    h[0] = st->e;
    h[1] = st->d;
    h[2] = st->ginv;
    h[3] = st->phi;
    h[4] = 1.0;
  }
  st->it += 1.0;
  st->oldb = oldb;
  st->beta = beta;
  st->s = beta > 0.0 ? 1.0 / beta : 0.0;
  st->c_r1 = beta > 0.0 ? -beta / oldb : 0.0;
  if (!(st->phibar > st->tol * st->beta1) || beta == 0.0 || !(alfa == alfa)) st->done = 1.0;
}

__global__ void k_ms_step(MinresState *st, double *hist, int B) {
  if (threadIdx.x || blockIdx.x) return;
  ms_step(st + blockIdx.y, hist + (int64_t)blockIdx.y * kMsRec * B, B);
}

// v = s y, also stored in slot st->slot of the Lanczos block vh (slot stride vs; the slot is
// clamped to [0, B - 1])
__global__ void k_ms_scale(double *v, const double *y, const MinresState *st, int64_t n, double *vh, int64_t vs,
                           int B) {
  const int64_t o = (int64_t)blockIdx.y * n;
  const double a = st[blockIdx.y].s;
  int sl = (int)st[blockIdx.y].slot;
  sl = sl < 0 ? 0 : sl >= B ? B - 1 : sl;
  double *h = vh + (int64_t)sl * vs + o;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double t = a * y[o + i];
    v[o + i] = t;
    h[i] = t;
  }
}

// y += c_r1 r1 - (alfa s) r2   (the second term after alfa is known: two launches)
__global__ void k_ms_axpy(double *y, const double *r, const MinresState *st, int which, int64_t n) {
  const MinresState &q = st[blockIdx.y];
  const double a = which == 0 ? q.c_r1 : -q.alfa * q.s;
  if (a == 0.0) return;
  const int64_t o = (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[o + i] += a * r[o + i];
}

// y -= (alfa s) r2 as k_ms_axpy (which = 1), then the FP32 copy of the first n32 entries
// of y for the FP32 preconditioner (lane stride l32)
__global__ void k_ms_axpy_f32(double *y, const double *r, const MinresState *st, int64_t n, float *y32, int64_t n32,
                              int64_t l32) {
  const MinresState &q = st[blockIdx.y];
  const double a = -q.alfa * q.s;
  const int64_t o = (int64_t)blockIdx.y * n;
  y32 += (int64_t)blockIdx.y * l32;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = y[o + i];
    if (a != 0.0) {
      v += a * r[o + i];
      y[o + i] = v;
    }
    if (i < n32) y32[i] = (float)v;
  }
}

// Coefficients of a block of m iterations (block = lane): the direction recurrence run on
// coefficient vectors over the basis (v slot 0 .. m - 1, w_{k0-1}, w_{k0}), stopping at the
// first slot the lane did not apply; thread k follows coefficient k (the recurrence acts on
// each coefficient alone).  Writes, per lane at coef + lane (1 + 3 (B + 2)): the number of
// applied slots, then the coefficients of the x increment, of the new w_{k-1} and of the new
// w_k (m + 2 each, at stride B + 2).  Resets the lane's slot.
__global__ void k_ms_coef(const double *hist, int B, int m, double *coef, MinresState *st) {
  const int lane = blockIdx.x, k = threadIdx.x, nb = m + 2;
  const double *h = hist + (int64_t)lane * kMsRec * B;
  double *cf = coef + (int64_t)lane * (1 + 3 * (B + 2));
  if (k < nb) {
    double w2 = k == m ? 1.0 : 0.0, w1 = k == m + 1 ? 1.0 : 0.0, cx = 0.0;
    int applied = 0;
    for (int i = 0; i < m; ++i) {
      const double *r = h + kMsRec * i;
      if (r[4] == 0.0) break;
      const double e = r[0], d = r[1], g = r[2], phi = r[3];
      const double wn = ((k == i ? 1.0 : 0.0) - e * w2 - d * w1) * g;
      cx += phi * wn;
      w2 = w1;
      w1 = wn;
      ++applied;
    }
    cf[1 + k] = cx;
    cf[1 + (B + 2) + k] = w2;
    cf[1 + 2 * (B + 2) + k] = w1;
    if (k == 0) {
      cf[0] = (double)applied;
      st[lane].slot = 0.0;
    }
  }
}

// x += the block's increment; unless last, w_{k-1} and w_k over W2 and W1 (in place: every
// output entry depends only on the same entry of the inputs).  first: x, W2 and W1 are zero
// and not read.  A lane with no applied slot is left as it is.  Sums in slot order, then
// W2, W1.
__global__ void k_ms_combine(double *x, double *W2, double *W1, const double *vh, int64_t vs, const double *coef,
                             int B, int m, int64_t n, int first, int last) {
  const double *cf = coef + (int64_t)blockIdx.y * (1 + 3 * (B + 2));
  const int ma = (int)cf[0];
  if (ma == 0) return;
  const double *cx = cf + 1, *ca = cf + 1 + (B + 2), *cb = cf + 1 + 2 * (B + 2);
  const int64_t o = (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double ax = first ? 0.0 : x[o + i], aa = 0.0, ab = 0.0;
    const double *p = vh + o + i;
    int k = 0;
    for (; k + 8 <= ma; k += 8) {   // eight independent loads in flight, sums in slot order
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u) * vs];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        ax += cx[k + u] * v[u];
        aa += ca[k + u] * v[u];
        ab += cb[k + u] * v[u];
      }
    }
    for (; k < ma; ++k) {
      const double v = p[(int64_t)k * vs];
      ax += cx[k] * v;
      aa += ca[k] * v;
      ab += cb[k] * v;
    }
    if (!first) {
      const double w2 = W2[o + i], w1 = W1[o + i];
      ax += cx[m] * w2 + cx[m + 1] * w1;
      aa += ca[m] * w2 + ca[m + 1] * w1;
      ab += cb[m] * w2 + cb[m + 1] * w1;
    }
    x[o + i] = ax;
    if (!last) {
      W2[o + i] = aa;
      W1[o + i] = ab;
    }
  }
}

// alfa = sum of the per-tile parts of v . y (one block per lane, fixed order)
__global__ void __launch_bounds__(1024) k_ms_alfa(const double *part, int n, MinresState *st) {
  __shared__ double red[1024 / kWave];
  part += (int64_t)blockIdx.y * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += part[i];
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int k = 0; k < 1024 / kWave; ++k) b += red[k];
    st[blockIdx.y].alfa = b;
  }
}

// beta^2 = the velocity tile sums, then the pressure block sums (one 1024-thread block per
// lane, fixed order; lane k's sums at part + k lp, its state at st + k), then the step
// (ms_step) of that lane
__global__ void __launch_bounds__(1024) k_ms_beta_step(const double *part, int nu, int np, int64_t lp,
                                                       MinresState *st, double *hist, int B) {
  __shared__ double red[1024 / kWave];
  part += (int64_t)blockIdx.y * lp;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nu + np; i += 1024) acc += part[i];
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int k = 0; k < 1024 / kWave; ++k) b += red[k];
    st[blockIdx.y].beta2 = b;
    ms_step(st + blockIdx.y, hist + (int64_t)blockIdx.y * kMsRec * B, B);
  }
}

// Buffers of one rotation phase (0, 1, 2).  Lanczos: r1 (old), r2 (current), y (new); v the
// scaled vector (assembled-A11 form; the matrix-free form writes it straight into the block);
// W2, W1 the directions w_{k0-1}, w_{k0} carried between blocks.  Lane 0 of each (lane
// stride nf).
struct MsBufs {
  double *v, *r1, *r2, *y, *W2, *W1, *x;
};

static MsBufs ms_bufs(Ctx &c, double *x, int phase) {
  double *B[3] = {c.inner.v64[2].p, c.inner.v64[3].p, c.inner.v64[1].p};   // r1, r2, y at phase 0
  MsBufs b;
  b.v = c.inner.v64[0].p;
  b.r1 = B[phase % 3];
  b.r2 = B[(phase + 1) % 3];
  b.y = B[(phase + 2) % 3];
  b.W2 = c.inner.v64[4].p;
  b.W1 = c.inner.v64[5].p;
  b.x = x;
  return b;
}

// Buffers with the matrix-free A11 product (fused iteration below): the new Lanczos vector
// is written over r1, so r1 and r2 alternate between two buffers and the preconditioned
// vector always lives in the third (period 2).
static MsBufs ms_bufs_fused(Ctx &c, double *x, int it) {
  MsBufs b = ms_bufs(c, x, 0);
  double *B0 = c.inner.v64[2].p, *B1 = c.inner.v64[3].p;
  b.r1 = it % 2 == 0 ? B0 : B1;
  b.r2 = it % 2 == 0 ? B1 : B0;
  b.y = c.inner.v64[1].p;
  return b;
}

// The preconditioner can hand over r . z as tile and block sums when the velocity cycle of
// its precision ends with the fused three-step launch on a matrix-free hierarchy of two or
// more levels (the FP32 form for one system, on FP64 vectors).
static bool tile_dot_ok(const Ctx &c, bool fp32) {
  return c.mgu.stencil && c.mgu.lv.size() > 1 && (fp32 ? c.mgu.degree32 : c.mgu.degree) == 3 && c.ms_dot.p;
}

// One inner iteration with the matrix-free A11 (FP64) for K systems: the scaling v = s y,
// the product, the first three-term update and the dot product alfa = v . y are one tiled
// launch (new y over r1); then y -= alfa s r2, z = M y into the y buffer, beta^2 = y . z.
template <typename TA>
static void ms_iteration_fused(Ctx &c, const MsBufs &b, MinresState *st, int K) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np;
  const unsigned g = vgrid(nf);
  double *dv = (double *)st;
  const int tiles = stencil_tile_count(c.n);
  stencil_a11_minres(c.n, (const StencilTable<double> *)c.mgu.lv[0].stab64.p, (const DivTable<double> *)c.divtab64.p,
                     LP<const double>(b.y, nf), LP<double>(c.ms_vh.p, nf), LP<double>(b.r1, nf),
                     LP<const double>(&st->s, kMsDoubles), LP<const double>(&st->c_r1, kMsDoubles),
                     LP<const double>(&st->slot, kMsDoubles), (int64_t)c.lanes * nf, c.ms_B,
                     LP<double>(c.ms_part.p, tiles), s, K);
  hipLaunchKernelGGL(k_ms_alfa, dim3(1, K), dim3(1024), 0, s, c.ms_part.p, tiles, st);
  constexpr bool f32 = std::is_same<TA, float>::value;
  const bool dot_ok = tile_dot_ok(c, f32);
  if (f32 && dot_ok)   // the three-term update also writes the FP32 copy the preconditioner reads
    hipLaunchKernelGGL(k_ms_axpy_f32, dim3(g, K), dim3(256), 0, s, b.r1, b.r2, st, nf, c.outer.x32.p,
                       K == 1 ? 2 * c.N2 : nf, nf);
  else
    hipLaunchKernelGGL(k_ms_axpy, dim3(g, K), dim3(256), 0, s, b.r1, b.r2, st, 1, nf);
  if (dot_ok) {   // beta^2 = r . z from the launches that write z
    const int nu = cheb3_dot_count(c.n), np = pres_dot_count(c);
    const int64_t ld = nu + pres_dot_slots(c.n);
    const LP<double> dot(c.ms_dot.p, ld);
    if constexpr (f32) {   // the same arithmetic as a11_precond_on64<float>, sums on FP64 r
      if (K == 1) {
        a11_precond<float>(c, c.outer.x32.p, nullptr, 1, b.r1, b.y, dot);
      } else {
        a11_precond<float>(c, c.outer.x32.p, c.outer.y32.p, K, b.r1, nullptr, dot);
        convert_l(LP<double>(b.y, nf), LP<const float>(c.outer.y32.p, nf), nf, s, K);
      }
    } else {
      a11_precond<double>(c, b.r1, b.y, K, nullptr, nullptr, dot);
    }
    hipLaunchKernelGGL(k_ms_beta_step, dim3(1, K), dim3(1024), 0, s, c.ms_dot.p, nu, np, ld, st,
                       c.ms_hist.p, c.ms_B);
  } else {
    a11_precond_on64<TA>(c, b.r1, b.y, K);
    dot_l(LP<const double>(b.r1, nf), LP<const double>(b.y, nf), nf, LP<double>(dv + 1, kMsDoubles), c.ms_red.p, s,
          K);
    hipLaunchKernelGGL(k_ms_step, dim3(1, K), dim3(1), 0, s, st, c.ms_hist.p, c.ms_B);
  }
  FSI_CHECK_LAUNCH();
}

// The same with the assembled A11 (one system)
template <typename TA>
static void ms_iteration(Ctx &c, const MsBufs &b, MinresState *st) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np;
  const unsigned g = vgrid(nf);
  double *dv = (double *)st;   // alfa at 0, beta2 at 1
  hipLaunchKernelGGL(k_ms_scale, dim3(g), dim3(256), 0, s, b.v, b.y, st, nf, c.ms_vh.p, (int64_t)c.lanes * nf,
                     c.ms_B);
  apply_a11_on64<double>(c, b.v, b.y);
  hipLaunchKernelGGL(k_ms_axpy, dim3(g), dim3(256), 0, s, b.y, b.r1, st, 0, nf);
  multidot(b.v, 0, 1, b.y, nf, dv, c.ms_red, s);
  hipLaunchKernelGGL(k_ms_axpy, dim3(g), dim3(256), 0, s, b.y, b.r2, st, 1, nf);
  // new Lanczos vector is b.y: precondition it into the buffer of r1 (no longer needed)
  a11_precond_on64<TA>(c, b.y, b.r1);
  multidot(b.y, 0, 1, b.r1, nf, dv + 1, c.ms_red, s);
  hipLaunchKernelGGL(k_ms_step, dim3(1), dim3(1), 0, s, st, c.ms_hist.p, c.ms_B);
  FSI_CHECK_LAUNCH();
}

// MINRES on K systems A11 x_k = b_k in lockstep (host arrays of K device vectors; K > 1
// needs the matrix-free A11).  Every system has its own scalar state and stops updating its
// x once converged; the loop ends when all have.  its[k] = iterations of system k.
template <typename TA>
static void minres_a11(Ctx &c, const double *const *b, double *const *xout, int K, double tol, int maxit,
                       int *its) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np;
  const bool fused = c.mgu.stencil;   // matrix-free FP64 A11
  FSI_REQUIRE(K >= 1 && K <= c.lanes, FSI_E_ARG, "more systems than inner lanes");
  FSI_REQUIRE(K == 1 || fused, FSI_E_STATE, "several systems per inner solve need the matrix-free smoother");
  MinresState *st = (MinresState *)c.ms_state.p;
  double *dv = (double *)st;
  double *x = c.ms_x.p;
  MsBufs b0 = ms_bufs(c, x, 0);
  fill_l(LP<double>(x, nf), nf, 0.0, s, K);
  // phase 0 expects: r2 = current Lanczos vector, y = M r2
  for (int k = 0; k < K; ++k) convert(b0.r2 + k * nf, b[k], nf, s);
  a11_precond_any<TA>(c, b0.r2, b0.y, K);
  dot_l(LP<const double>(b0.r2, nf), LP<const double>(b0.y, nf), nf, LP<double>(dv + 1, kMsDoubles), c.ms_red.p, s,
        K);
  hipLaunchKernelGGL(k_ms_init, dim3(1, K), dim3(1), 0, s, st, tol);
  FSI_CHECK_LAUNCH();
  const bool graphs = c.use_graphs && !(c.prof64.on || c.prof32.on);
  // with graphs the state is read back every second step (a replay costs far more than the
  // read-back; checking every 8 steps measured 5-12% slower at 64^2 and 128^2 from the
  // frozen steps run past convergence)
  const int check_every = graphs ? 2 : 1;
  // Lagged check (eager launches; by default on grids of n <= kMsLagMaxN): the state of step
  // it - 1 is read back after step it has been enqueued (a copy and an event per step, two
  // host buffers), so the device does not wait for the host between steps; the step enqueued
  // past convergence is frozen by the done flag, which costs one step per solve.  On larger
  // grids a step takes long enough that the wait is the smaller cost.
  const bool lag = !graphs && (c.ms_check == FSI_CHECK_LAGGED ||
                               (c.ms_check == FSI_CHECK_AUTO && c.n <= kMsLagMaxN));
  const int pk = std::is_same<TA, double>::value ? 0 : 1;
  int it = 0, k0 = 0;   // iterations done; iterations before the current block
  const int B = c.ms_B;
  // x (and, unless last, the carried directions) from the block of iterations k0 .. it - 1
  auto flush = [&](bool last) {
    const int m = it - k0;
    if (m == 0) return;
    hipLaunchKernelGGL(k_ms_coef, dim3(K), dim3(kWave), 0, s, c.ms_hist.p, B, m, c.ms_coef.p, st);
    hipLaunchKernelGGL(k_ms_combine, dim3((unsigned)((nf + 255) / 256), K), dim3(256), 0, s, x, b0.W2, b0.W1,
                       c.ms_vh.p, (int64_t)c.lanes * nf, c.ms_coef.p, B, m, nf, k0 == 0 ? 1 : 0, last ? 1 : 0);
    FSI_CHECK_LAUNCH();
    k0 = it;
  };
  double *h = c.hpin;
  static_assert(FSI_MAX_LANES * kMsDoubles <= kHpinHalf, "two state copies in the pinned buffer");
  auto states_done = [&](const double *hb) {
    bool done = true;
    for (int k = 0; k < K; ++k) {
      const MinresState *hs = (const MinresState *)hb + k;
      FSI_REQUIRE(hs->phibar == hs->phibar && hs->beta == hs->beta, FSI_E_NONFINITE,
                  "non-finite value in the inner A11 solve");
      done = done && hs->done != 0.0;
    }
    return done;
  };
  auto all_done = [&]() {
    FSI_HIP(hipMemcpyAsync(h, st, (size_t)K * kMsDoubles * sizeof(double), hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    return states_done(h);
  };
  while (it < maxit) {
    // the rotation: in phase p the roles are shifted by p (r2 of phase p is y of p-1, ...)
    const int phase = fused ? it % 2 : it % 3;
    const MsBufs bq = fused ? ms_bufs_fused(c, x, it) : ms_bufs(c, x, phase);
    if (graphs) {
      hipGraphExec_t &ge = c.ms_graph[pk][K][phase];
      if (!ge)
        capture_graph(c, ge, [&] {
          if (fused) ms_iteration_fused<TA>(c, bq, st, K);
          else ms_iteration<TA>(c, bq, st);
        });
      FSI_HIP(hipGraphLaunch(ge, s));
    } else if (fused) {
      ms_iteration_fused<TA>(c, bq, st, K);
    } else {
      ms_iteration<TA>(c, bq, st);
    }
    ++it;
    if (it - k0 == B) flush(false);
    if (lag) {
      double *hb = h + (it & 1) * kHpinHalf;
      FSI_HIP(hipMemcpyAsync(hb, st, (size_t)K * kMsDoubles * sizeof(double), hipMemcpyDeviceToHost, s));
      FSI_HIP(hipEventRecord(c.ev_ms[it & 1], s));
      if (it >= 2) {   // step it - 1, while step it runs
        FSI_HIP(hipEventSynchronize(c.ev_ms[(it - 1) & 1]));
        if (states_done(h + ((it - 1) & 1) * kHpinHalf)) break;
      }
    } else if ((it % check_every == 0 || it == maxit) && all_done()) {
      break;
    }
  }
  flush(true);
  all_done();
  for (int k = 0; k < K; ++k) {
    const MinresState *hs = (const MinresState *)h + k;
    its[k] = (int)hs->it;
    convert(xout[k], x + k * nf, nf, s);
    if (trace_on())
      std::fprintf(stderr, "[fsi] minres<%s> lane=%d/%d its=%d relres_est=%.3e beta=%.3e graphs=%d\n",
                   std::is_same<TA, double>::value ? "f64" : "f32", k, K, its[k],
                   hs->beta1 > 0 ? hs->phibar / hs->beta1 : 0.0, hs->beta, graphs ? 1 : 0);
  }
}

// The fixed-cost inexact A11^{-1} of K systems (host arrays of device vectors): one
// application of the MINRES preconditioner diag(MG(A_f), S~^{-1}), with the pressure part
// negated (A11 = [A_f -B^T; -B 0] has the Schur complement -B A_f^{-1} B^T) except the pinned
// entry, whose row of A11 is the identity.
template <typename TA>
static void a11_fixed(Ctx &c, const double *const *r, double *const *z, int K) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np, nv = 2 * c.N2 + 1;
  const MsBufs b0 = ms_bufs(c, c.ms_x.p, 0);
  for (int k = 0; k < K; ++k) convert(b0.r2 + k * nf, r[k], nf, s);
  a11_precond_any<TA>(c, b0.r2, b0.y, K);
  for (int k = 0; k < K; ++k) {
    convert(z[k], b0.y + k * nf, nv, s);
    hipLaunchKernelGGL(k_negate<double>, dim3(vgrid(nf - nv)), dim3(256), 0, s, z[k] + nv, b0.y + k * nf + nv,
                       nf - nv);
  }
  FSI_CHECK_LAUNCH();
}

// The fixed-cost block-triangular A11^{-1} (FSI_INNER_FIXED_TRI): `cycles` steps of the stationary
// iteration z <- z + P^{-1} (r - A11 z) from z = 0 with the block upper-triangular
// approximation of A11 = [A_f, -B^T; -B, 0] (pinned row: the identity),
//   P = [V^{-1}, -B^T; 0, -S~]:  z_p = -S~^{-1} r_p (the pinned entry: r_p),
//                                z_u = V (r_u + B^T z_p),
// V one velocity V-cycle and S~^{-1} the Cahouet-Chabard approximation of the MINRES
// preconditioner.  With exact blocks every eigenvalue of P^{-1} A11 is 1 (the block
// factorisation of A11), so the iteration converges; the block-diagonal form does not (its
// preconditioned A11 has the eigenvalues 1 and (1 +- i sqrt 3) / 2).  The pressure part
// runs before the velocity cycle, on one stream.
template <typename TA>
static void a11_tri_apply(Ctx &c, const double *r, double *z, double *q, double *y, int K) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np, nv = 2 * c.N2 + 1;
  a11_precond_on64<TA>(c, r, z, K, PC_PRES);   // z_p = S~^{-1} r_p, z_p[pin] = r_p[pin]
  for (int k = 0; k < K; ++k) {
    double *zk = z + k * nf, *qk = q + k * nf;
    hipLaunchKernelGGL(k_negate<double>, dim3(vgrid(nf - nv)), dim3(256), 0, s, zk + nv, zk + nv, nf - nv);
    // r_u + B^T z_p = r_u - (A11 [0; z_p])_u
    fill(qk, 2 * c.N2, 0.0, s);
    convert(qk + 2 * c.N2, zk + 2 * c.N2, c.Np, s);
    apply_a11_on64<double>(c, qk, y + k * nf);
  }
  lincomb_l(LP<double>(q, nf), LP<const double>(r, nf), LP<const double>(y, nf), 1.0, -1.0, 2 * c.N2, s, K);
  a11_precond_on64<TA>(c, q, z, K, PC_VEL);    // z_u = V (r_u + B^T z_p)
  FSI_CHECK_LAUNCH();
}

template <typename TA>
static void a11_fixed_tri(Ctx &c, const double *const *r, double *const *z, int K, int cycles) {
  hipStream_t s = c.stream;
  const int64_t nf = 2 * c.N2 + c.Np;
  double *R = c.inner.v64[2].p, *Z = c.inner.v64[3].p, *T = c.inner.v64[4].p, *D = c.inner.v64[5].p;
  double *Q = c.inner.v64[0].p, *Y = c.inner.v64[1].p;
  for (int k = 0; k < K; ++k) convert(R + k * nf, r[k], nf, s);
  a11_tri_apply<TA>(c, R, Z, Q, Y, K);
  for (int cyc = 1; cyc < cycles; ++cyc) {
    for (int k = 0; k < K; ++k) apply_a11_on64<double>(c, Z + k * nf, Y + k * nf);
    lincomb_l(LP<double>(T, nf), LP<const double>(R, nf), LP<const double>(Y, nf), 1.0, -1.0, nf, s, K);
    a11_tri_apply<TA>(c, T, D, Q, Y, K);
    lincomb_l(LP<double>(Z, nf), LP<const double>(Z, nf), LP<const double>(D, nf), 1.0, 1.0, nf, s, K);
  }
  for (int k = 0; k < K; ++k) convert(z[k], Z + k * nf, nf, s);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- A22 closed form (FP64)
// C_s^{-1} by Chebyshev-Jacobi steps on the interval [1/2, 2] of D^{-1} C_s (P1 mass matrix on
// triangles): the error falls by 1/3 per step, and 36 steps reach the rounding level
// ((1/3)^36 < 1e-17), so A22 is inverted exactly in FP64 as the method asks (an inexact A22 is
// the harmful one, Sec. 7).  Measured at 1024^2 / 256^2 / 512^2: taking the solve only four
// orders below the inner tolerance (12-13 steps) left every outer and inner step count
// unchanged and saved 2% of the step; the exact form is kept.
static int cs_steps(const Ctx &c) { return c.cs_nsteps; }

static const double *cs_solve(Ctx &c, const double *b, double *scratch, int steps) {
  const int64_t ns = c.Ns;
  double *t = scratch, *t2 = t + 2 * ns, *d = t + 4 * ns;
  return chebyshev<double, 1, 2>(ns, c.S.rowptr.p, c.S.col.p, c.Cs.p, c.Cs_dinv.p, c.cs_lo, c.cs_hi,
                                 steps, b, t, t2, d, true, c.stream);
}

// The same closed form for every system of a batch in one launch: one 1024-thread block per
// system.  A_s and C_s act on each component alone, so the two components run one after the
// other: the iterate of the current Chebyshev solve lies in LDS as two buffers of Ns entries
// (read one, write the other), a thread's rows (at most kA22Rows) keep their right-hand side
// and direction in registers, and the rows of A_s and C_s come from device memory in the
// transposed layout (entry u of row r at u Ns + r: the lanes of a wave, consecutive rows,
// read consecutive words; the row-major CSR made every load of a wave touch a dozen or more
// cache lines).  Same steps as a22_solve: t = C_s^{-1} r_lam, z_X = -dt t,
// u = r_X - A_s z_X, z_lam = -C_s^{-1} u.
constexpr int kA22Threads = 1024, kA22Rows = 7, kA22Nnz = 7;
struct A22Lane {
  const int *rp, *ecol;            // CSR row pointer (row lengths); transposed columns
  const double *eas, *ecs, *csd;   // A_s and C_s values (transposed); C_s inverse diagonal
  const double *rX, *rl;
  double *zX, *zl;
  int ns;
  double dt;
};
struct A22Args {
  A22Lane lane[FSI_MAX_LANES];
  int steps;
  double theta, delta;             // Chebyshev interval of D^{-1} C_s: centre and half width
};

// s[q] = sum over the len[q] entries of row tid + kA22Threads q (in CSR order) of val x[col]
// in the transposed layout (row stride ns): entry u of every row of the thread at a time (one
// uniform base per entry, the loads of all rows issued together), the entries beyond
// kA22Nnz (rare on a triangle mesh) in order after them
__device__ __forceinline__ void a22_rows(const int *ecol, const double *eval, const double *x, int tid, int ns,
                                         const int (&len)[kA22Rows], double (&s)[kA22Rows]) {
#pragma unroll
  for (int q = 0; q < kA22Rows; ++q) s[q] = 0.0;
#pragma unroll
  for (int u = 0; u < kA22Nnz; ++u) {
    const int *cu = ecol + (size_t)u * ns;
    const double *vu = eval + (size_t)u * ns;
#pragma unroll
    for (int q = 0; q < kA22Rows; ++q) {
      const unsigned r = (unsigned)(tid + kA22Threads * q);
      if (u < len[q]) s[q] += vu[r] * x[cu[r]];
    }
  }
#pragma unroll
  for (int q = 0; q < kA22Rows; ++q) {
    const size_t r = (size_t)(tid + kA22Threads * q);
    for (int u = kA22Nnz; u < len[q]; ++u) s[q] += eval[(size_t)u * ns + r] * x[ecol[(size_t)u * ns + r]];
  }
}

__global__ void __launch_bounds__(kA22Threads) k_a22_lanes(A22Args a) {
  extern __shared__ double a22_x[];   // two buffers of ns entries
  const A22Lane &L = a.lane[blockIdx.y];
  const int ns = L.ns, tid = threadIdx.x;
  int len[kA22Rows];                  // lengths of this thread's rows (the pattern of both matrices)
#pragma unroll
  for (int q = 0; q < kA22Rows; ++q) {
    const int r = tid + kA22Threads * q;
    len[q] = r < ns ? L.rp[r + 1] - L.rp[r] : 0;
  }
  // C_s^{-1} b by the Chebyshev steps of chebyshev<double, 1, 2> from zero (b: this thread's
  // rows); returns the buffer holding the result
  auto cs_solve = [&](const double (&b)[kA22Rows]) -> double * {
    const double sigma = a.theta / a.delta;
    double rho = 1.0 / sigma;
    double d[kA22Rows];
    double *x = a22_x, *x2 = a22_x + ns;
#pragma unroll
    for (int q = 0; q < kA22Rows; ++q) {
      const int r = tid + kA22Threads * q;
      if (r < ns) {
        const double z = 1.0 / a.theta * L.csd[r] * b[q];
        d[q] = z;
        x[r] = z;
      }
    }
    __syncthreads();
    for (int k = 1; k < a.steps; ++k) {
      const double rho1 = 1.0 / (2.0 * sigma - rho);
      const double c1 = rho1 * rho, c2 = 2.0 * rho1 / a.delta;
      rho = rho1;
      // the row stride, opaque to the compiler within the step: the entry addresses are
      // formed in the step instead of being held, all of them, across the steps
      int nss = ns;
      asm volatile("" : "+s"(nss));
      double sr[kA22Rows];
      a22_rows(L.ecol, L.ecs, x, tid, nss, len, sr);
#pragma unroll
      for (int q = 0; q < kA22Rows; ++q) {
        const int r = tid + kA22Threads * q;
        if (r < ns) {
          const double s0 = sr[q];
          d[q] = c1 * d[q] + c2 * (L.csd[r] * (b[q] - s0));
          x2[r] = x[r] + d[q];
        }
      }
      __syncthreads();
      double *t = x;
      x = x2;
      x2 = t;
    }
    return x;
  };
  for (int c = 0; c < 2; ++c) {
    const int64_t o = (int64_t)c * ns;
    double b[kA22Rows];
#pragma unroll
    for (int q = 0; q < kA22Rows; ++q) {
      const int r = tid + kA22Threads * q;
      b[q] = r < ns ? L.rl[o + r] : 0.0;
    }
    double *t = cs_solve(b);
    // z_X = -dt t (stored; kept in the other buffer for the A_s rows)
    double *zx = t == a22_x ? a22_x + ns : a22_x;
#pragma unroll
    for (int q = 0; q < kA22Rows; ++q) {
      const int r = tid + kA22Threads * q;
      if (r < ns) {
        const double tv = t[r];
        const double z = -L.dt * tv + 0.0 * tv;
        L.zX[o + r] = z;
        zx[r] = z;
      }
    }
    __syncthreads();
    // u = r_X - A_s z_X
    {
      double sr[kA22Rows];
      a22_rows(L.ecol, L.eas, zx, tid, ns, len, sr);
#pragma unroll
      for (int q = 0; q < kA22Rows; ++q) {
        const int r = tid + kA22Threads * q;
        if (r < ns) b[q] = L.rX[o + r] - sr[q];
      }
    }
    __syncthreads();   // every row has read z_X: the next solve starts over both buffers
    const double *t2 = cs_solve(b);
#pragma unroll
    for (int q = 0; q < kA22Rows; ++q) {
      const int r = tid + kA22Threads * q;
      if (r < ns) L.zl[o + r] = -t2[r];
    }
    __syncthreads();   // the buffers are free for the next component
  }
}

// LDS grant of the batched closed form (device limit, at most 160 KiB), set once
static int a22_lds_limit() {
  static int limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    v = v < 65536 ? v : v > 163840 ? 163840 : v;
    if (v > 65536 &&
        hipFuncSetAttribute((const void *)k_a22_lanes, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) {
      (void)hipGetLastError();
      v = 65536;
    }
    return v;
  }();
  return limit;
}

// Whether a system's solid block fits the one-launch form
static bool a22_fits(const Ctx &c) {
  return c.Ns >= 1 && c.Ns <= (int64_t)kA22Threads * kA22Rows && c.s_ecol.p && c.s_ew >= 1 &&
         (int64_t)2 * c.Ns * (int64_t)sizeof(double) <= a22_lds_limit();   // two buffers of Ns
}

// z2 = A22^{-1} r2 on [X | lam] (4 Ns entries)
static void a22_solve(Ctx &c, const double *rX, const double *rl, double *zX, double *zl, int steps) {
  hipStream_t s = c.stream;
  const int64_t ns = c.Ns;
  double *scr = c.tmpS.p, *u = c.tmpS.p + 6 * ns;
  const double *t = cs_solve(c, rl, scr, steps);
  lincomb(zX, t, t, -c.dt, 0.0, 2 * ns, s);
  // u = r_X - A_s z_X;  z_lam = C_s^{-1} (A_s z_X - r_X) = -C_s^{-1} u  (the tangent of the
  // nonlinear solid in place of A_s while it is set: 2 x 2 blocks)
  if (c.use_kt) spmv<double, 4, 2, SP_RESID>(ns, c.S.rowptr.p, c.S.col.p, c.Kt.p, zX, ns, u, ns, s, rX);
  else spmv<double, 1, 2, SP_RESID>(ns, c.S.rowptr.p, c.S.col.p, c.S.val.p, zX, ns, u, ns, s, rX);
  const double *t2 = cs_solve(c, u, scr, steps);
  hipLaunchKernelGGL(k_negate<double>, dim3(vgrid(2 * ns)), dim3(256), 0, s, zl, t2, 2 * ns);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- block preconditioner
// Inner work space for K systems: the MINRES vectors and state, the V-cycle level vectors
// and the staging of the captured preconditioner hold c.lanes systems each (lane stride =
// one system's length).  Growing the lane count reallocates them and drops the captured
// graphs (they hold the old addresses).
static void ensure_inner(Ctx &c, int prec, int K = 1) {
  FSI_REQUIRE(K >= 1 && K <= FSI_MAX_LANES, FSI_E_ARG, "lane count out of range");
  const int64_t nf = 2 * c.N2 + c.Np;
  if (K > c.lanes) {
    FSI_HIP(hipStreamSynchronize(c.stream));   // captured graphs may still be running
    c.drop_graphs();
    for (int i = 0; i < 9; ++i) {
      c.inner.v64[i].release();
      c.inner.v32[i].release();
    }
    for (auto *b : {&c.ms_x, &c.ms_state, &c.ms_red, &c.ms_part, &c.ms_dot, &c.pc_in, &c.pc_out, &c.ms_vh,
                    &c.ms_hist, &c.ms_coef})
      b->release();
    c.outer.x32.release();
    c.outer.y32.release();
    for (Mg *mg : {&c.mgu, &c.mgp})
      for (auto &L : mg->lv)
        for (int i = 0; i < 5; ++i) {
          L.w64[i].alloc((size_t)K * mg->comps * L.nodes);
          L.w32[i].release();   // reallocated at the new size by ensure_fp32_mg
        }
    c.lanes = K;
  }
  const int64_t nl = c.lanes;
  for (int i = 0; i < 9; ++i)
    if (!c.inner.v64[i].p) c.inner.v64[i].alloc(nl * nf);
  if (!c.ms_vh.p) {   // Lanczos block: at most kMsBMax vectors per lane, 2 GiB over all lanes
    const int64_t fit = (int64_t(2) << 30) / (8 * nl * nf);
    c.ms_B = (int)std::max<int64_t>(4, std::min<int64_t>(kMsBMax, fit));
    c.ms_vh.alloc((size_t)c.ms_B * nl * nf);
    c.ms_hist.alloc((size_t)nl * kMsRec * c.ms_B);
    c.ms_coef.alloc((size_t)nl * (1 + 3 * (c.ms_B + 2)));
  }
  if (!c.ms_x.p) {
    c.ms_x.alloc(nl * nf);
    c.ms_state.alloc(nl * kMsDoubles);
    c.ms_red.alloc(nl * red_blocks(nf));   // dot products of one system per lane: never regrown
    c.ms_part.alloc(nl * stencil_tile_count(c.n));
    c.ms_dot.alloc(nl * (cheb3_dot_count(c.n) + pres_dot_slots(c.n)));
  }
  if (!c.pc_in.p) {
    c.pc_in.alloc(nl * nf);
    c.pc_out.alloc(nl * nf);
  }
  if (prec == FSI_FP32) {
    ensure_fp32_mg(c);
    for (int i = 7; i < 9; ++i)       // pressure scratch of the FP32 preconditioner
      if (!c.inner.v32[i].p) c.inner.v32[i].alloc(nl * nf);
    if (!c.outer.x32.p) { c.outer.x32.alloc(nl * nf); c.outer.y32.alloc(nl * nf); }
    if (!c.Mp_dinv32.p) {
      c.Mp_dinv32.alloc(c.Np);
      convert(c.Mp_dinv32.p, c.Mp_dinv.p, c.Np, c.stream);
    }
  }
}

// Default inner tolerance (flexible outer GMRES: it trades outer for inner steps).
// Block-triangular: 1e-2 in both precisions.  Measured on the 1024^2 / 256^2 / 512^2
// workloads with the multigrid of this file, FP64 step time at 1.5e-3, 3e-3, 6e-3, 1e-2,
// 2e-2: 247/235/203/193/225, 138/137/117/106/103, 60/55/51/48/54 ms (outer steps 9, 10, 5 up
// to 1e-2, one more at 2e-2 on two workloads); mixed at 5e-3, 1e-2, 2e-2, 4e-2:
// 182/152/177/142, 104/97/94/95, 46/42/47/45 ms.  Its outer counts equal the exact-block
// counts (10, 11, 14 at 32^2, 128^2, 256^2) at 1e-2 already.
// Block-diagonal: 1e-6.  Its outer counts react much more to the inexact A11.  Against the
// exact-block counts 16 / 16 / 20 (random right-hand sides at 32^2 / 128^2 / 256^2) and 4 (the
// first step of the rotating disk at 256^2) it takes 16 / 18 / 22 / 8 at 1e-3, 16 / 16 / 20 / 6
// at 1e-4 and 1e-5, and 16 / 16 / 20 / 4 at 1e-6.  Time at 1e-6 against 1e-3: +23%, +23%,
// +25% on the random right-hand sides, -27% on the time step.
// Weight of the pressure rows in the residual norm of the inner GMRES: the ratio of the scales
// of the two diagonal blocks of the block-diagonal approximation diag(A_f^{-1}, S~^{-1}), so
// that ||D r|| behaves like the norm MINRES uses.  w = sqrt(a_u s_p): a_u the mean diagonal of
// A_f at interior nodes (the four classes' 2 x 2 blocks), s_p = nu / m_p + (rho/dt) / l_p with
// m_p and l_p the interior diagonals of the P1 mass and Laplacian (the Cahouet-Chabard
// scale).  About 2 n with nu = 1, rho/dt = 100.  Without it (w = 1) the inner solves at 1e-2
// leave the divergence rows, whose entries are O(h) times smaller, nearly unconverged: at
// 128^2 the step at rtol 1e-8 was 3.5e-7 (u) and 1.3e-6 (p) away from the oracle, against
// 1.5e-9 and 5.6e-9 with w = n (4 n and 16 n: the same errors, more inner steps).
double inner_pressure_weight(Ctx &c) {
  if (c.gi_wp > 0) return c.gi_wp;
  StencilTable<double> a;
  StencilTable<float> af;
  stencil_tables(c.n, c.nu, c.rho / c.dt, a, af);
  double au = 0.0;
  for (int k = 0; k < 4; ++k) {   // the diagonal of the inverse of each class's D^{-1} block
    const double *d = a.dinv[k];
    const double det = d[0] * d[3] - d[1] * d[2];
    au += 0.25 * 0.5 * (d[0] + d[3]) / det;
  }
  P1Table<double> mp, lp;
  P1Table<float> f;
  p1_tables(c.n, kTableMp, 0, mp, f);
  p1_tables(c.n, kTableLp, 0, lp, f);
  const double sp = c.nu * mp.dinv[4] + (c.rho / c.dt) * lp.dinv[4];
  FSI_REQUIRE(au > 0 && sp > 0, FSI_E_STATE, "non-positive diagonal scales");
  c.gi_wp = std::sqrt(au * sp);
  return c.gi_wp;
}

// The paper's element pair, block-triangular: 1e-4.  Its pressure slopes leave little trace in
// the outer residual, so looser inner solves stop the outer iteration with the pressure far from
// the solution: the 32^2 bar's step at rtol 1e-8 was 3.9e-7 (p) from the oracle's direct solve at
// 1e-2, 1.9e-7 at 1e-3 and 1.7e-9 (the oracle's exact-block GMRES: 1.6e-9) at 1e-4, with 76 /
// 101 / 122 inner steps.
double inner_tol(const Ctx &c, int prec, int pc) {
  (void)prec;
  if (c.inner_rtol > 0) return c.inner_rtol;
  if (pc == FSI_PC_DIAG) return 1e-6;
  return c.pair == FSI_PAIR_Q2P1DISC ? 1e-4 : 1e-2;
}

template <typename TA>
static void gmres_a11(Ctx &c, const double *const *b, double *const *xout, int K, double tol, int maxit, int *its);

// The block preconditioner on K systems: system k belongs to context cs[k] (one fluid grid
// and fluid parameters for all); the A11 solves of all run in lockstep on the inner lanes of
// the engine context c (one of them or another of the same grid) with its inner and smoother
// settings, then each system's A22 part on its own context.  Every context's stream must be
// c's for the call.
void apply_precond_lanes(Ctx &c, Ctx *const *cs, int K, int pc, int prec, const double *const *r,
                         double *const *z) {
  FSI_REQUIRE(pc == FSI_PC_DIAG || pc == FSI_PC_TRI, FSI_E_ARG, "unknown preconditioner");
  FSI_REQUIRE(prec == FSI_FP64 || prec == FSI_FP32 || prec == FSI_FP32_IR, FSI_E_ARG,
              "unknown precision");
  if (prec == FSI_FP32_IR) prec = FSI_FP32;
  for (int k = 0; k < K; ++k)
    FSI_REQUIRE(cs[k]->have_cf || pc == FSI_PC_DIAG, FSI_E_STATE,
                "block-triangular needs C_f: call fsi_assemble_coupling");
  ensure_inner(c, prec, K);
  const double tol = inner_tol(c, prec, pc);
  int its[FSI_MAX_LANES];
  if (c.inner_mode == FSI_INNER_FIXED_DIAG) {   // one application of the MINRES preconditioner
    if (prec == FSI_FP64) a11_fixed<double>(c, r, z, K);
    else a11_fixed<float>(c, r, z, K);
    for (int k = 0; k < K; ++k) its[k] = 0;
  } else if (c.inner_mode == FSI_INNER_FIXED_TRI) {   // block-triangular stationary cycles
    if (prec == FSI_FP64) a11_fixed_tri<double>(c, r, z, K, c.inner_cycles);
    else a11_fixed_tri<float>(c, r, z, K, c.inner_cycles);
    for (int k = 0; k < K; ++k) its[k] = 0;
  } else if (c.inner_mode == FSI_INNER_GMRES) {   // GMRES, block-triangular approximation
    if (prec == FSI_FP64) gmres_a11<double>(c, r, z, K, tol, c.inner_maxit, its);
    else gmres_a11<float>(c, r, z, K, tol, c.inner_maxit, its);
  } else if (prec == FSI_FP64) {   // the default: MINRES, block-diagonal SPD preconditioner
    minres_a11<double>(c, r, z, K, tol, c.inner_maxit, its);
  } else {
    minres_a11<float>(c, r, z, K, tol, c.inner_maxit, its);
  }
  // the solid blocks: every system's closed form in one launch when all fit, else one by one.
  // The one-workgroup form serves the 36-step mass solves of P1 solids; for the 56 steps of Q1
  // solids the launches over the whole GPU measured faster (256^2 bar, 2,781 solid nodes: 102.4
  // against 109.5 ms per FP64 step)
  bool fit = true;
  int ns_max = 0;
  for (int k = 0; k < K; ++k) {
    fit = fit && a22_fits(*cs[k]) && !cs[k]->use_kt && cs[k]->cs_nsteps <= 36 && cs[k]->cs_lo == cs[0]->cs_lo &&
          cs[k]->cs_hi == cs[0]->cs_hi && cs[k]->cs_nsteps == cs[0]->cs_nsteps;
    ns_max = std::max(ns_max, (int)cs[k]->Ns);
  }
  A22Args aa{};
  for (int k = 0; k < K; ++k) {
    Ctx &ck = *cs[k];
    ck.inner_its_total += its[k];
    hipStream_t s = ck.stream;
    const int64_t nf = 2 * ck.N2 + ck.Np, ns = ck.Ns;
    const double *rX = r[k] + nf, *rl = r[k] + nf + 2 * ns;
    double *zX = z[k] + nf, *zl = z[k] + nf + 2 * ns;
    if (pc == FSI_PC_TRI) {
      // r_lam - C_f z_u  (A21 z1 = [0; C_f z_u])
      double *t = ck.tmpS.p + 8 * ns;
      spmv<double, 1, 2, SP_RESID>(ns, ck.Cf.rowptr.p, ck.Cf.col.p, ck.Cf.val.p, z[k], ck.N2, t, ns, s, rl);
      rl = t;
    }
    if (fit)
      aa.lane[k] = A22Lane{ck.S.rowptr.p, ck.s_ecol.p, ck.s_eas.p, ck.s_ecs.p, ck.Cs_dinv.p, rX, rl, zX, zl, (int)ns,
                           ck.dt};
    else
      a22_solve(ck, rX, rl, zX, zl, cs_steps(ck));
  }
  if (fit) {
    aa.steps = cs_steps(*cs[0]);
    aa.theta = 0.5 * (cs[0]->cs_hi + cs[0]->cs_lo);   // the C_s interval of cs_solve
    aa.delta = 0.5 * (cs[0]->cs_hi - cs[0]->cs_lo);
    hipLaunchKernelGGL(k_a22_lanes, dim3(1, (unsigned)K), dim3(kA22Threads), (size_t)2 * ns_max * sizeof(double),
                       c.stream, aa);
    FSI_CHECK_LAUNCH();
  }
}

void apply_precond(Ctx &c, int pc, int prec, const double *r, double *z) {
  Ctx *cs[1] = {&c};
  apply_precond_lanes(c, cs, 1, pc, prec, &r, &z);
}

// ---------------------------------------------------------------- outer FGMRES
static void op_apply(Ctx &c, int prec, const double *x, double *y) {
  if (prec == FSI_FP64) apply_operator<double, double>(c, x, y, false);
  else apply_operator<float, double>(c, x, y, false);
}

// r = b - A x (FP64)
static void residual64(Ctx &c, const double *b, const double *x, double *r) {
  apply_operator<double, double>(c, x, r, false);
  axpby(r, b, 1.0, -1.0, c.N, c.stream);
}

// The Gram-Schmidt reductions of one Arnoldi step for every system of a batch in one launch
// each (lane = blockIdx.y): the same partition, order and arithmetic as multidot and
// k_multiaxpy_sub on one system (red_blocks(n) chunks of the lane's own length), so each
// system's numbers do not depend on the batch.
struct ArnLane {
  const double *V;   // Krylov basis (k vectors at stride ldv, n when ldv is 0)
  const double *w;   // current vector (w for the dots, updated in place by the axpy)
  double *part;      // red_blocks(n) * k partial sums
  double *h;         // k results
  int64_t n;
  int k, nb;
  int64_t ldv;
};
struct ArnArgs {
  ArnLane l[FSI_MAX_LANES];
};

// this thread's parts of V_q . w for G vectors V_q = v + q n over the chunk [lo, hi) (G a
// compile-time count: no branch between the loads, which issue together)
template <int G>
__device__ __forceinline__ void arn_dot_group(const double *v, const double *w, int64_t ldv, int64_t lo, int64_t hi,
                                              double (&s)[4]) {
#pragma unroll 4
  for (int64_t e = lo + threadIdx.x; e < hi; e += kRedBlock) {
    const double we = w[e];
#pragma unroll
    for (int q = 0; q < G; ++q) s[q] += v[(int64_t)q * ldv + e] * we;
  }
}

__global__ void __launch_bounds__(kRedBlock) k_arn_dot_part(ArnArgs a) {
  const ArnLane &L = a.l[blockIdx.y];
  if ((int)blockIdx.x >= L.nb) return;
  const int64_t chunk = (L.n + L.nb - 1) / L.nb;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < L.n ? lo + chunk : L.n;
  // four basis vectors per pass over the chunk: w is read once per group and the four
  // block sums share one barrier; every sum keeps the order of a single dot product
  constexpr int G = 4;
  __shared__ double ws[G][kRedBlock / kWave];
  const int64_t ldv = L.ldv ? L.ldv : L.n;
  for (int i0 = 0; i0 < L.k; i0 += G) {
    const int g = L.k - i0 < G ? L.k - i0 : G;   // uniform over the block
    const double *v = L.V + (int64_t)i0 * ldv;
    double s[G] = {0.0, 0.0, 0.0, 0.0};
    switch (g) {
      case 4: arn_dot_group<4>(v, L.w, ldv, lo, hi, s); break;
      case 3: arn_dot_group<3>(v, L.w, ldv, lo, hi, s); break;
      case 2: arn_dot_group<2>(v, L.w, ldv, lo, hi, s); break;
      default: arn_dot_group<1>(v, L.w, ldv, lo, hi, s); break;
    }
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const double t = wave_sum(s[q]);
      if (lane == 0) ws[q][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < g) {
      double t = 0.0;
      for (int k = 0; k < kRedBlock / kWave; ++k) t += ws[threadIdx.x][k];
      L.part[(int64_t)(i0 + threadIdx.x) * L.nb + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

__global__ void k_arn_dot_final(ArnArgs a) {
  const ArnLane &L = a.l[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= L.k) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < L.nb; b += kWave) s += L.part[(int64_t)i * L.nb + b];
  s = wave_sum(s);
  if (threadIdx.x == 0) L.h[i] = s;
}

__global__ void k_arn_axpy_sub(ArnArgs a) {   // w -= sum_i h[i] V_i
  const ArnLane &L = a.l[blockIdx.y];
  double *w = const_cast<double *>(L.w);
  const int64_t ldv = L.ldv ? L.ldv : L.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L.n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = w[e];
    for (int i = 0; i < L.k; ++i) s -= L.h[i] * L.V[(int64_t)i * ldv + e];
    w[e] = s;
  }
}

static void arn_dots(ArnArgs &a, int K, int kmax, int nbmax, hipStream_t s) {
  hipLaunchKernelGGL(k_arn_dot_part, dim3((unsigned)nbmax, (unsigned)K), dim3(kRedBlock), 0, s, a);
  hipLaunchKernelGGL(k_arn_dot_final, dim3((unsigned)kmax, (unsigned)K), dim3(kWave), 0, s, a);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- inner GMRES on A11
// A11^{-1} of K systems (FSI_INNER_GMRES) by right-preconditioned restarted GMRES with
// the block upper-triangular approximation P of a11_tri_apply (one cycle, a fixed linear
// operator) to ||D (b - A11 x)|| <= tol ||D b||, from x = 0, with D = diag(I, w I) weighting
// the pressure rows (inner_pressure_weight): GMRES runs on D A11 D^{-1} with the
// preconditioner D P^{-1} D^{-1}.  The spectrum of P^{-1} A11 is that of the Schur
// approximation's S~^{-1} S (real, in (0, 1]) perturbed by the velocity cycle, where a Krylov
// method gains far more per step than the stationary cycles and than MINRES with the
// block-diagonal preconditioner (which must treat both signs of the saddle-point spectrum).
// Arnoldi with two classical Gram-Schmidt passes (the kernels of the outer solve); the
// Hessenberg least-squares problem on the host, one synchronisation per step for all
// systems.  Basis V_j and preconditioned vectors Z_j = P^{-1} V_j of all lanes stored
// [j][lane][nf]; x += Z y once a lane converges or its cycle ends.  Every lane follows its
// own sequence of operations, so its result does not depend on the batch.
constexpr int kGiM = 20;   // inner restart length

__global__ void k_lane_scale(double *v, const double *w, const double *scale, int64_t n) {
  const double a = scale[blockIdx.y];
  const int64_t o = (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[o + i] = a * w[o + i];
}

// dst = src with entries [off, n) of every lane scaled by a (dst may be src)
__global__ void k_lane_scale_tail(double *dst, const double *src, int64_t n, int64_t off, double a) {
  const int64_t o = (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[o + i] = i >= off ? a * src[o + i] : src[o + i];
}

// x_lane += sum_{i < count} y_i Z_i (lane's coefficients at coef + lane cs: count, y_0, ...)
__global__ void k_lane_combine(double *x, const double *Z, int64_t ldz, const double *coef, int cs, int64_t n) {
  const double *cf = coef + (int64_t)blockIdx.y * cs;
  const int cnt = (int)cf[0];
  if (cnt == 0) return;
  const int64_t o = (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double a = x[o + i];
    for (int k = 0; k < cnt; ++k) a += cf[1 + k] * Z[(int64_t)k * ldz + o + i];
    x[o + i] = a;
  }
}

double inner_pressure_weight(Ctx &c);

template <typename TA>
static void gmres_a11(Ctx &c, const double *const *b, double *const *xout, int K, double tol, int maxit, int *its) {
  hipStream_t s = c.stream;
  const double wp = inner_pressure_weight(c);
  const int64_t nf = 2 * c.N2 + c.Np, L = c.lanes, ld = L * nf;
  const int m = std::max(1, std::min(kGiM, maxit));
  const int nb = red_blocks(nf), st = 2 * (m + 1) + 1, cs = m + 1;
  c.gi_V.reserve((size_t)(m + 1) * ld);
  c.gi_Z.reserve((size_t)m * ld);
  c.gi_part.reserve((size_t)L * nb * (m + 1));
  c.gi_dh.reserve((size_t)L * st);
  c.gi_sc.reserve((size_t)L * (cs + 1));
  if (!c.gi_h) FSI_HIP(hipHostMalloc((void **)&c.gi_h, (size_t)FSI_MAX_LANES * (st + cs + 1) * 2 * sizeof(double),
                                     hipHostMallocDefault));
  double *hd = c.gi_h;                                       // device -> host results
  double *hu = c.gi_h + (size_t)FSI_MAX_LANES * (st + cs + 1);   // host -> device scalars
  double *X = c.inner.v64[3].p, *Bv = c.inner.v64[2].p, *R = c.inner.v64[4].p;
  double *Q = c.inner.v64[0].p, *Y = c.inner.v64[1].p;
  double *V = c.gi_V.p, *Z = c.gi_Z.p, *scale = c.gi_sc.p, *coef = c.gi_sc.p + L;
  fill_l(LP<double>(X, nf), nf, 0.0, s, K);
  for (int k = 0; k < K; ++k) convert(Bv + k * nf, b[k], nf, s);
  const int64_t pofs = 2 * c.N2;   // the pressure rows, weighted by wp in the residual norm
  auto weigh = [&](double *dst, const double *src, double a) {
    hipLaunchKernelGGL(k_lane_scale_tail, dim3(vgrid(nf), K), dim3(256), 0, s, dst, src, nf, pofs, a);
  };
  // per-lane norms (or h columns) of the vectors w_q: k = 1 dots into gi_dh + q st + off
  auto norms = [&](const double *w, int off) {
    ArnArgs a{};
    for (int q = 0; q < K; ++q)
      a.l[q] = ArnLane{w + q * nf, w + q * nf, c.gi_part.p + (int64_t)q * nb * (m + 1), c.gi_dh.p + q * st + off, nf,
                       1, nb, 0};
    arn_dots(a, K, 1, nb, s);
  };
  auto fetch = [&]() {
    FSI_HIP(hipMemcpyAsync(hd, c.gi_dh.p, (size_t)K * st * sizeof(double), hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
  };
  // the H2D copies read hu asynchronously: it is rewritten only after a later synchronisation
  auto scale_lanes = [&](double *dst, const double *src, const std::vector<double> &a) {
    for (int q = 0; q < K; ++q) hu[q] = a[q];
    FSI_HIP(hipMemcpyAsync(scale, hu, (size_t)K * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_lane_scale, dim3(vgrid(nf), K), dim3(256), 0, s, dst, src, scale, nf);
  };
  weigh(R, Bv, wp);
  norms(R, 2 * (m + 1));
  fetch();
  std::vector<double> bnorm(K), beta(K), sc(K);
  std::vector<int> done(K, 0), total(K, 0);
  for (int q = 0; q < K; ++q) {
    const double b2 = hd[q * st + 2 * (m + 1)];
    FSI_REQUIRE(std::isfinite(b2), FSI_E_NONFINITE, "non-finite right-hand side of the inner A11 solve");
    bnorm[q] = std::sqrt(b2 > 0 ? b2 : 0.0);
    done[q] = bnorm[q] == 0.0;
    beta[q] = bnorm[q];
  }
  std::vector<double> H((size_t)K * (m + 1) * m), gs((size_t)K * (m + 1)), cosv((size_t)K * m), sinv((size_t)K * m);
  std::vector<int> steps(K), act(K);
  bool first = true;
  auto any = [](const std::vector<int> &v) {
    for (int x : v) if (x) return true;
    return false;
  };
  while (true) {
    for (int q = 0; q < K; ++q) act[q] = !done[q] && total[q] < maxit;
    if (!any(act)) break;
    // V_0 = r / ||r||, r = D (b - A11 x) (D b on the first cycle)
    const double *r0 = R;
    if (!first) {
      for (int q = 0; q < K; ++q) apply_a11_on64<double>(c, X + q * nf, Y + q * nf);
      lincomb_l(LP<double>(R, nf), LP<const double>(Bv, nf), LP<const double>(Y, nf), 1.0, -1.0, nf, s, K);
      weigh(R, R, wp);
      norms(R, 2 * (m + 1));
      fetch();
      for (int q = 0; q < K; ++q) {
        const double r2 = hd[q * st + 2 * (m + 1)];
        FSI_REQUIRE(std::isfinite(r2), FSI_E_NONFINITE, "non-finite residual in the inner A11 solve");
        beta[q] = std::sqrt(r2 > 0 ? r2 : 0.0);
        if (act[q] && beta[q] <= tol * bnorm[q]) { act[q] = 0; done[q] = 1; }
      }
      if (!any(act)) break;
    }
    first = false;
    for (int q = 0; q < K; ++q) {
      sc[q] = act[q] && beta[q] > 0 ? 1.0 / beta[q] : 0.0;
      std::fill(gs.begin() + (size_t)q * (m + 1), gs.begin() + (size_t)(q + 1) * (m + 1), 0.0);
      gs[(size_t)q * (m + 1)] = beta[q];
      steps[q] = 0;
    }
    scale_lanes(V, r0, sc);
    std::vector<int> run = act;   // lanes still stepping in this cycle
    for (int j = 0; j < m && any(run); ++j) {
      double *Vj = V + (int64_t)j * ld, *Zj = Z + (int64_t)j * ld, *W = V + (int64_t)(j + 1) * ld;
      weigh(R, Vj, 1.0 / wp);   // Z_j = P^{-1} D^{-1} V_j, W = D A11 Z_j
      a11_tri_apply<TA>(c, R, Zj, Q, Y, K);
      for (int q = 0; q < K; ++q) apply_a11_on64<double>(c, Zj + q * nf, W + q * nf);
      weigh(W, W, wp);
      ArnArgs a1{}, a2{};
      for (int q = 0; q < K; ++q) {
        double *part = c.gi_part.p + (int64_t)q * nb * (m + 1), *dh = c.gi_dh.p + q * st;
        a1.l[q] = ArnLane{V + q * nf, W + q * nf, part, dh, nf, j + 1, nb, ld};
        a2.l[q] = ArnLane{V + q * nf, W + q * nf, part, dh + (m + 1), nf, j + 1, nb, ld};
      }
      arn_dots(a1, K, j + 1, nb, s);
      hipLaunchKernelGGL(k_arn_axpy_sub, dim3(vgrid(nf), (unsigned)K), dim3(256), 0, s, a1);
      arn_dots(a2, K, j + 1, nb, s);
      hipLaunchKernelGGL(k_arn_axpy_sub, dim3(vgrid(nf), (unsigned)K), dim3(256), 0, s, a2);
      norms(W, 2 * (m + 1));
      FSI_CHECK_LAUNCH();
      fetch();
      for (int q = 0; q < K; ++q) {
        sc[q] = 0.0;
        if (!run[q]) continue;
        const double *hp = hd + q * st;
        double *hc = &H[((size_t)q * m + j) * (m + 1)];   // column j of lane q
        for (int i = 0; i <= j; ++i) hc[i] = hp[i] + hp[(m + 1) + i];
        const double hn = std::sqrt(hp[2 * (m + 1)] > 0 ? hp[2 * (m + 1)] : 0.0);
        FSI_REQUIRE(std::isfinite(hn), FSI_E_NONFINITE, "non-finite vector in the inner A11 solve");
        hc[j + 1] = hn;
        double *cq = &cosv[(size_t)q * m], *sq = &sinv[(size_t)q * m], *g = &gs[(size_t)q * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double t = cq[i] * hc[i] + sq[i] * hc[i + 1];
          hc[i + 1] = -sq[i] * hc[i] + cq[i] * hc[i + 1];
          hc[i] = t;
        }
        const double den = std::hypot(hc[j], hc[j + 1]);
        cq[j] = den > 0 ? hc[j] / den : 1.0;
        sq[j] = den > 0 ? hc[j + 1] / den : 0.0;
        hc[j] = den;
        hc[j + 1] = 0.0;
        g[j + 1] = -sq[j] * g[j];
        g[j] = cq[j] * g[j];
        steps[q] = j + 1;
        ++total[q];
        const bool conv = std::fabs(g[j + 1]) <= tol * bnorm[q] || hn == 0.0;
        if (conv) done[q] = 1;
        if (conv || total[q] >= maxit) run[q] = 0;
        else sc[q] = 1.0 / hn;
      }
      if (j + 1 < m && any(run)) scale_lanes(W, W, sc);
    }
    // x += Z y for every lane that stepped in this cycle, y from the triangular system
    for (int q = 0; q < K; ++q) {
      double *cf = hu + K + (size_t)q * cs;
      const int k = act[q] ? steps[q] : 0;
      cf[0] = (double)k;
      const double *g = &gs[(size_t)q * (m + 1)];
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < k; ++l) t -= H[((size_t)q * m + l) * (m + 1) + i] * cf[1 + l];
        const double d = H[((size_t)q * m + i) * (m + 1) + i];
        cf[1 + i] = d != 0.0 ? t / d : 0.0;
      }
    }
    FSI_HIP(hipMemcpyAsync(coef, hu + K, (size_t)K * cs * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_lane_combine, dim3(vgrid(nf), K), dim3(256), 0, s, X, Z, ld, coef, cs, nf);
    FSI_CHECK_LAUNCH();
    FSI_HIP(hipStreamSynchronize(s));   // hu is reused by the next cycle
  }
  for (int k = 0; k < K; ++k) {
    its[k] = total[k];
    convert(xout[k], X + k * nf, nf, s);
  }
}

// One system of a lockstep FGMRES solve: its context, vectors, statistics and the state
// of its current restart cycle.
struct GmLane {
  Ctx *c = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
  fsi_solve_stats S{};
  double bnorm = 0.0, target = 0.0, rn = 0.0;
  enum { RESID, CYCLE, DONE } state = RESID;
  int rc = FSI_OK;
  std::string err;
  // restart cycle: Hessenberg columns (rotated), Givens rotations, rotated right-hand side
  std::vector<double> H, cs, sn, g;
  int j = 0, maxsteps = 0;
  double est = 0.0, cyc_target = 0.0;
  void fail(int code, const char *msg) {
    rc = code;
    err = msg;
    state = DONE;
  }
};

// FGMRES on K systems in lockstep (system k on context cs[k]: same fluid grid, parameters and
// options for all; every call runs on cs[0]'s stream, and cs[0] holds the inner lanes).  Each system follows exactly the
// sequence of operations of a solve on its own: restarted cycles of at most `restart`
// Arnoldi steps, each with the block preconditioner (all systems' A11 solves batched) and
// the FP64 or FP32 operator, modified Gram-Schmidt done twice, Givens rotations on the host;
// a system leaves the batch when its true residual meets rtol or its step budget is spent.
// rc[k] = FSI_OK, FSI_E_NOCONV or FSI_E_NONFINITE (msg in cs[k]->last_error).
void gmres_solve_lanes(Ctx *const *cs, int K, const fsi_solve_opts &o, const double *const *b,
                       double *const *x, fsi_solve_stats *st, int *rc) {
  Ctx &c0 = *cs[0];
  hipStream_t s = c0.stream;
  FSI_REQUIRE(K >= 1 && K <= FSI_MAX_LANES, FSI_E_ARG, "lane count out of range");
  const int m = o.restart > 0 ? o.restart : 30;
  FSI_REQUIRE(m <= 200, FSI_E_ARG, "restart length above 200");
  const int maxit = o.maxit > 0 ? o.maxit : 10000;
  const double rtol = o.rtol > 0 ? o.rtol : 1e-8;
  const int prec = o.prec;
  FSI_REQUIRE(prec == FSI_FP64 || prec == FSI_FP32 || prec == FSI_FP32_IR, FSI_E_ARG,
              "unknown precision");
  // operator of the Arnoldi process and arithmetic of the preconditioner
  const int op_prec = prec == FSI_FP32_IR ? FSI_FP32 : FSI_FP64;
  const int pc_prec = prec == FSI_FP64 ? FSI_FP64 : FSI_FP32;
  const bool refine = prec == FSI_FP32_IR;
  const double cyc = o.cycle_rtol > 0 ? o.cycle_rtol : 1e-5;
  // per-solve inner settings; each context's own (fsi_set_inner) come back afterwards
  struct Restore {
    Ctx *c;
    double r;
    int m, mode, cycles;
    ~Restore() {
      c->inner_rtol = r;
      c->inner_maxit = m;
      c->inner_mode = mode;
      c->inner_cycles = cycles;
    }
  };
  std::vector<Restore> restore;
  restore.reserve(K);
  std::vector<GmLane> L(K);
  for (int k = 0; k < K; ++k) {
    Ctx &c = *cs[k];
    FSI_REQUIRE(c.have_cf, FSI_E_STATE, "the solve needs C_f: call fsi_assemble_coupling first");
    FSI_REQUIRE(c.stream == s, FSI_E_STATE, "systems of one lockstep solve share one stream");
    FSI_REQUIRE(o.inner_mode >= FSI_INNER_MINRES && o.inner_mode <= FSI_INNER_GMRES, FSI_E_ARG,
                "unknown inner mode");
    FSI_REQUIRE(o.inner_cycles >= 0 && o.inner_cycles <= 100, FSI_E_ARG, "inner cycles out of range");
    restore.push_back({&c, c.inner_rtol, c.inner_maxit, c.inner_mode, c.inner_cycles});
    c.inner_mode = o.inner_mode;
    c.inner_cycles = o.inner_cycles > 0 ? o.inner_cycles : 1;
    if (o.inner_rtol > 0) c.inner_rtol = o.inner_rtol;
    if (o.inner_maxit > 0) c.inner_maxit = o.inner_maxit;
    else if (prec == FSI_FP32) c.inner_maxit = std::min(c.inner_maxit, 300);
    const int64_t N = c.N;
    if (c.outer.m < m || c.outer.ncap < N) {
      const int mm = std::max(m, c.outer.m);
      const int64_t nn = std::max(N, c.outer.ncap);
      c.outer.V.alloc((size_t)(mm + 1) * nn);
      c.outer.Z.alloc((size_t)mm * nn);
      c.outer.m = mm;
      c.outer.ncap = nn;
    }
    c.outer.w.reserve(N);
    c.outer.r.reserve(N);
    c.dscal.reserve(8 + 2 * (m + 1) + 1 + 64);
    c.red.reserve((size_t)red_blocks(N) * (m + 1));   // Gram-Schmidt partial sums: no regrowth mid-solve
    c.inner_its_total = 0;
    L[k].c = &c;
    L[k].b = b[k];
    L[k].x = x[k];
    L[k].H.assign((size_t)(m + 1) * m, 0.0);
    L[k].cs.assign(m, 0.0);
    L[k].sn.assign(m, 0.0);
    L[k].g.assign(m + 1, 0.0);
  }
  // ||b||: one dot product per system, one synchronisation for all
  for (auto &l : L) {
    multidot(l.b, 0, 1, l.b, l.c->N, l.c->dscal.p, l.c->red, s);
    FSI_HIP(hipMemcpyAsync(l.c->hpin, l.c->dscal.p, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  FSI_HIP(hipStreamSynchronize(s));
  for (auto &l : L) {
    l.bnorm = std::sqrt(l.c->hpin[0]);
    if (!std::isfinite(l.bnorm)) {
      l.fail(FSI_E_NONFINITE, "non-finite right-hand side");
    } else if (l.bnorm == 0.0) {
      fill(l.x, l.c->N, 0.0, s);
      l.S.converged = 1;
      l.state = GmLane::DONE;
    }
    l.target = rtol * l.bnorm;
  }
  std::vector<Ctx *> pcs;
  std::vector<const double *> pr;
  std::vector<double *> pz;
  while (true) {
    // true residuals of the systems between cycles
    bool any = false;
    for (auto &l : L)
      if (l.state == GmLane::RESID) {
        Ctx &c = *l.c;
        residual64(c, l.b, l.x, c.outer.r.p);
        multidot(c.outer.r.p, 0, 1, c.outer.r.p, c.N, c.dscal.p, c.red, s);
        FSI_HIP(hipMemcpyAsync(c.hpin, c.dscal.p, sizeof(double), hipMemcpyDeviceToHost, s));
        any = true;
      }
    if (any) FSI_HIP(hipStreamSynchronize(s));
    for (auto &l : L) {
      if (l.state != GmLane::RESID) continue;
      Ctx &c = *l.c;
      l.rn = std::sqrt(c.hpin[0]);
      if (!std::isfinite(l.rn)) { l.fail(FSI_E_NONFINITE, "non-finite residual"); continue; }
      if (l.rn <= l.target) { l.S.converged = 1; l.state = GmLane::DONE; continue; }
      if (l.S.its >= maxit) { l.fail(FSI_E_NOCONV, "GMRES reached maxit"); continue; }
      // a cycle toward the final target; with FP32_IR, refinement cycles that each ask the
      // FP32 operator for a cycle_rtol reduction of the FP64 residual
      l.cyc_target = refine ? std::max(l.target, cyc * l.rn) : l.target;
      l.maxsteps = maxit - l.S.its;
      std::fill(l.H.begin(), l.H.end(), 0.0);
      std::fill(l.g.begin(), l.g.end(), 0.0);
      l.g[0] = l.rn;
      l.j = 0;
      l.est = l.rn;
      lincomb(c.outer.V.p, c.outer.r.p, c.outer.r.p, 1.0 / l.rn, 0.0, c.N, s);
      l.state = GmLane::CYCLE;
    }
    // one Arnoldi step of every system inside a cycle
    pcs.clear();
    pr.clear();
    pz.clear();
    for (auto &l : L)
      if (l.state == GmLane::CYCLE) {
        Ctx &c = *l.c;
        pcs.push_back(&c);
        pr.push_back(c.outer.V.p + (int64_t)l.j * c.N);
        pz.push_back(c.outer.Z.p + (int64_t)l.j * c.N);
      }
    if (pcs.empty()) break;
    apply_precond_lanes(c0, pcs.data(), (int)pcs.size(), o.pc, pc_prec, pr.data(), pz.data());
    // the operator of every system, then classical Gram-Schmidt twice and the norm of w for
    // all systems at once (h1 at 0, h2 at m + 1, |w|^2 at 2 (m + 1) of each system's slot),
    // copied to the host in one transfer
    const int stride = 2 * (m + 1) + 1;
    std::vector<GmLane *> act;
    for (auto &l : L)
      if (l.state == GmLane::CYCLE) act.push_back(&l);
    const int KA = (int)act.size();
    c0.bat_dh.reserve((size_t)KA * stride);
    if (c0.bat_h_n < (size_t)KA * stride) {
      if (c0.bat_h) FSI_HIP(hipHostFree(c0.bat_h));
      c0.bat_h = nullptr;
      c0.bat_h_n = 0;
      FSI_HIP(hipHostMalloc((void **)&c0.bat_h, (size_t)FSI_MAX_LANES * stride * sizeof(double),
                            hipHostMallocDefault));
      c0.bat_h_n = (size_t)FSI_MAX_LANES * stride;
    }
    ArnArgs a1{}, a2{}, a3{};
    int kmax = 1, nbmax = 1;
    int64_t nmax = 1;
    for (int q = 0; q < KA; ++q) {
      Ctx &c = *act[q]->c;
      const int64_t N = c.N;
      const int j = act[q]->j, nb = red_blocks(N);
      op_apply(c, op_prec, c.outer.Z.p + (int64_t)j * N, c.outer.w.p);
      c.red.reserve((size_t)nb * (j + 1));
      double *dh = c0.bat_dh.p + (int64_t)q * stride;
      a1.l[q] = ArnLane{c.outer.V.p, c.outer.w.p, c.red.p, dh, N, j + 1, nb};
      a2.l[q] = ArnLane{c.outer.V.p, c.outer.w.p, c.red.p, dh + (m + 1), N, j + 1, nb};
      a3.l[q] = ArnLane{c.outer.w.p, c.outer.w.p, c.red.p, dh + 2 * (m + 1), N, 1, nb};
      kmax = std::max(kmax, j + 1);
      nbmax = std::max(nbmax, nb);
      nmax = std::max(nmax, N);
    }
    arn_dots(a1, KA, kmax, nbmax, s);
    hipLaunchKernelGGL(k_arn_axpy_sub, dim3(vgrid(nmax), (unsigned)KA), dim3(256), 0, s, a1);
    arn_dots(a2, KA, kmax, nbmax, s);
    hipLaunchKernelGGL(k_arn_axpy_sub, dim3(vgrid(nmax), (unsigned)KA), dim3(256), 0, s, a2);
    arn_dots(a3, KA, 1, nbmax, s);
    FSI_CHECK_LAUNCH();
    FSI_HIP(hipMemcpyAsync(c0.bat_h, c0.bat_dh.p, (size_t)KA * stride * sizeof(double), hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < KA; ++q) {
      GmLane &l = *act[q];
      Ctx &c = *l.c;
      const int64_t N = c.N;
      const int j = l.j;
      const double *hp = c0.bat_h + (int64_t)q * stride;
      double *hcol = &l.H[(size_t)j * (m + 1)];   // column j, rows 0..j+1
      for (int i = 0; i <= j; ++i) hcol[i] = hp[i] + hp[(m + 1) + i];
      const double hn = std::sqrt(hp[2 * (m + 1)] > 0 ? hp[2 * (m + 1)] : 0.0);
      if (!std::isfinite(hn)) { l.fail(FSI_E_NONFINITE, "non-finite Arnoldi vector"); continue; }
      hcol[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double t = l.cs[i] * hcol[i] + l.sn[i] * hcol[i + 1];
        hcol[i + 1] = -l.sn[i] * hcol[i] + l.cs[i] * hcol[i + 1];
        hcol[i] = t;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      l.cs[j] = hcol[j] / den;
      l.sn[j] = hcol[j + 1] / den;
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      l.g[j + 1] = -l.sn[j] * l.g[j];
      l.g[j] = l.cs[j] * l.g[j];
      l.est = std::fabs(l.g[j + 1]);
      const int k = j + 1;
      if (!(l.est <= l.cyc_target || hn == 0.0 || k >= l.maxsteps || k >= m)) {
        lincomb(c.outer.V.p + (int64_t)k * N, c.outer.w.p, c.outer.w.p, 1.0 / hn, 0.0, N, s);
        l.j = k;
        continue;
      }
      // end of the cycle: back substitution H y = g, x += Z y
      std::vector<double> y(k, 0.0);
      for (int i = k - 1; i >= 0; --i) {
        double t = l.g[i];
        for (int q = i + 1; q < k; ++q) t -= l.H[(size_t)q * (m + 1) + i] * y[q];
        y[i] = t / l.H[(size_t)i * (m + 1) + i];
      }
      // hpin holds y until the copy has run: it is rewritten only after a later synchronisation
      for (int i = 0; i < k; ++i) c.hpin[i] = y[i];
      double *dh = c.dscal.p + 8;
      FSI_HIP(hipMemcpyAsync(dh, c.hpin, k * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_multiaxpy_add, dim3(vgrid(N)), dim3(256), 0, s, l.x, c.outer.Z.p, N, k, dh, N);
      FSI_CHECK_LAUNCH();
      if (trace_on())
        std::fprintf(stderr, "[fsi] cycle prec=%d steps=%d rn/bn=%.3e est/bn=%.3e\n", prec, k, l.rn / l.bnorm,
                     l.est / l.bnorm);
      l.S.its += k;
      l.S.restarts += 1;
      if (refine) l.S.refinements += 1;
      l.S.relres_est = l.est / l.bnorm;
      l.state = GmLane::RESID;
    }
  }
  FSI_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < K; ++k) {
    GmLane &l = L[k];
    if (l.bnorm > 0.0 && std::isfinite(l.bnorm)) l.S.relres_true = l.rn / l.bnorm;
    l.S.inner_its = l.c->inner_its_total;
    if (st) st[k] = l.S;
    rc[k] = l.rc;
    if (l.rc != FSI_OK) l.c->last_error = l.err;
  }
}

void gmres_solve(Ctx &c, const fsi_solve_opts &o, const double *b, double *x, fsi_solve_stats *st) {
  Ctx *cs[1] = {&c};
  int rc = FSI_OK;
  fsi_solve_stats S{};
  gmres_solve_lanes(cs, 1, o, &b, &x, &S, &rc);
  if (st) *st = S;
  if (rc != FSI_OK) throw Error(rc, c.last_error);
}

}  // namespace fsi
