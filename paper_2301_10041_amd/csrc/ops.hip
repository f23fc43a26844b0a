// The operator of eq. (matrix) (Sec. 4) as one fused launch over three row groups, and
// the right-hand side (g1, 0, 0, g2).
//
//   velocity rows (P2 node r):  y_u = A_f x_u - B^T x_p + C_f^T x_lam
//   pressure rows (P1 node k):  y_p = -B x_u (+ x_p at the pinned node 0)
//   solid rows (node l):        y_X = A_s x_X - C_s x_lam,  y_lam = C_f x_u - (1/dt) C_s x_X
//
// G = 4 lanes per row; the row groups are separate ranges of blocks so every branch is
// uniform over a block.  T is the arithmetic (and value) type, Tx the input vector type
// and Ty the output type, so the FP32 form reads FP64 or FP32 vectors, computes and
// accumulates in FP32, and writes either.  With `fluid_only` the launch is the operator
// A11 on [u | p] (the C_f^T term and the solid rows are skipped).
#include "ctx.h"
#include "kernels.h"
#include "stencil.h"

namespace fsi {

constexpr int kG = 4;
constexpr int kOpBlock = 256;
constexpr int kRowsPerBlock = kOpBlock / kG;

template <typename T, typename Tx, typename Ty>
struct OpArgs {
  int64_t N2, Np, Ns;
  T inv_dt;
  // A_f (width 4), B^T (width 2), C_f^T (width 1)
  const int *af_rp, *af_col; const T *af_val;
  const int *bt_rp, *bt_col; const T *bt_val;
  const int *cft_rp, *cft_col; const T *cft_val;
  // B (width 2)
  const int *b_rp, *b_col; const T *b_val;
  // solid pattern: A_s, C_s; C_f
  const int *s_rp, *s_col; const T *as_val, *cs_val;
  const T *kt_val;   // non-null: the solid tangent (2 x 2 blocks) in place of A_s
  const int *cf_rp, *cf_col; const T *cf_val;
  const Tx *x;
  Ty *y;
  unsigned gU, gP;
  int fluid_only;
};

template <typename T, typename Tx, typename Ty>
__global__ void __launch_bounds__(kOpBlock) k_operator(OpArgs<T, Tx, Ty> a) {
  const int lane = threadIdx.x % kG;
  const int64_t N2 = a.N2, Np = a.Np, Ns = a.Ns;
  const Tx *xux = a.x, *xuy = a.x + N2, *xp = a.x + 2 * N2;
  const Tx *xXx = xp + Np, *xXy = xXx + Ns, *xlx = xXy + Ns, *xly = xlx + Ns;
  unsigned blk = blockIdx.x;
  if (blk < a.gU) {
    int64_t r = (int64_t)blk * kRowsPerBlock + threadIdx.x / kG;
    if (r >= N2) return;
    T sx = 0, sy = 0;
    for (int k = a.af_rp[r] + lane; k < a.af_rp[r + 1]; k += kG) {
      int j = a.af_col[k];
      const T *v = a.af_val + 4 * (int64_t)k;
      T x0 = (T)xux[j], x1 = (T)xuy[j];
      sx += v[0] * x0 + v[1] * x1;
      sy += v[2] * x0 + v[3] * x1;
    }
    for (int k = a.bt_rp[r] + lane; k < a.bt_rp[r + 1]; k += kG) {
      T pj = (T)xp[a.bt_col[k]];
      sx -= a.bt_val[2 * (int64_t)k] * pj;
      sy -= a.bt_val[2 * (int64_t)k + 1] * pj;
    }
    if (!a.fluid_only) {
      for (int k = a.cft_rp[r] + lane; k < a.cft_rp[r + 1]; k += kG) {
        int j = a.cft_col[k];
        T c = a.cft_val[k];
        sx += c * (T)xlx[j];
        sy += c * (T)xly[j];
      }
    }
    sx = group_sum<kG>(sx);
    sy = group_sum<kG>(sy);
    if (lane == 0) {
      a.y[r] = (Ty)sx;
      a.y[N2 + r] = (Ty)sy;
    }
    return;
  }
  blk -= a.gU;
  if (blk < a.gP) {
    int64_t r = (int64_t)blk * kRowsPerBlock + threadIdx.x / kG;
    if (r >= Np) return;
    T s = 0;
    for (int k = a.b_rp[r] + lane; k < a.b_rp[r + 1]; k += kG) {
      int j = a.b_col[k];
      s -= a.b_val[2 * (int64_t)k] * (T)xux[j] + a.b_val[2 * (int64_t)k + 1] * (T)xuy[j];
    }
    s = group_sum<kG>(s);
    if (lane == 0) a.y[2 * N2 + r] = (Ty)(r == 0 ? s + (T)xp[0] : s);
    return;
  }
  blk -= a.gP;
  int64_t l = (int64_t)blk * kRowsPerBlock + threadIdx.x / kG;
  if (l >= Ns) return;
  T aXx = 0, aXy = 0, cLx = 0, cLy = 0, cXx = 0, cXy = 0, fx = 0, fy = 0;
  for (int k = a.s_rp[l] + lane; k < a.s_rp[l + 1]; k += kG) {
    int j = a.s_col[k];
    T cs = a.cs_val[k];
    T Xx = (T)xXx[j], Xy = (T)xXy[j];
    if (a.kt_val) {
      const T *kt = a.kt_val + 4 * (int64_t)k;
      aXx += kt[0] * Xx + kt[1] * Xy;
      aXy += kt[2] * Xx + kt[3] * Xy;
    } else {
      T as = a.as_val[k];
      aXx += as * Xx; aXy += as * Xy;
    }
    cXx += cs * Xx; cXy += cs * Xy;
    cLx += cs * (T)xlx[j]; cLy += cs * (T)xly[j];
  }
  for (int k = a.cf_rp[l] + lane; k < a.cf_rp[l + 1]; k += kG) {
    int j = a.cf_col[k];
    T c = a.cf_val[k];
    fx += c * (T)xux[j];
    fy += c * (T)xuy[j];
  }
  aXx = group_sum<kG>(aXx); aXy = group_sum<kG>(aXy);
  cLx = group_sum<kG>(cLx); cLy = group_sum<kG>(cLy);
  cXx = group_sum<kG>(cXx); cXy = group_sum<kG>(cXy);
  fx = group_sum<kG>(fx); fy = group_sum<kG>(fy);
  if (lane == 0) {
    Ty *yX = a.y + 2 * N2 + Np;
    yX[l] = (Ty)(aXx - cLx);
    yX[Ns + l] = (Ty)(aXy - cLy);
    yX[2 * Ns + l] = (Ty)(fx - a.inv_dt * cXx);
    yX[3 * Ns + l] = (Ty)(fy - a.inv_dt * cXy);
  }
}

template <typename T>
static const T *vals(const Csr &A);
template <>
const double *vals<double>(const Csr &A) { return A.val.p; }
template <>
const float *vals<float>(const Csr &A) { return A.val32.p; }

void make_shadow(Csr &A, hipStream_t s) {
  size_t m = (size_t)A.nnz * A.width;
  A.val32.reserve(m);
  convert(A.val32.p, A.val.p, (int64_t)m, s);
}

// solid_only: only the solid row group (the fluid rows come from the stencil launch)
template <typename T, typename Tx, typename Ty>
static void launch_operator(Ctx &c, const Tx *x, Ty *y, bool fluid_only, bool solid_only = false) {
  OpArgs<T, Tx, Ty> a{};
  a.N2 = c.N2; a.Np = c.Np; a.Ns = fluid_only ? 0 : c.Ns;
  a.inv_dt = (T)(1.0 / c.dt);
  a.af_rp = c.Af.rowptr.p; a.af_col = c.Af.col.p; a.af_val = vals<T>(c.Af);
  a.bt_rp = c.BT.rowptr.p; a.bt_col = c.BT.col.p; a.bt_val = vals<T>(c.BT);
  a.b_rp = c.B.rowptr.p; a.b_col = c.B.col.p; a.b_val = vals<T>(c.B);
  if (!fluid_only) {
    a.cft_rp = c.CfT.rowptr.p; a.cft_col = c.CfT.col.p; a.cft_val = vals<T>(c.CfT);
    a.s_rp = c.S.rowptr.p; a.s_col = c.S.col.p; a.as_val = vals<T>(c.S);
    a.cs_val = std::is_same<T, double>::value ? (const T *)c.Cs.p : (const T *)c.Cs32.p;
    a.kt_val = !c.use_kt ? nullptr : std::is_same<T, double>::value ? (const T *)c.Kt.p : (const T *)c.Kt32.p;
    a.cf_rp = c.Cf.rowptr.p; a.cf_col = c.Cf.col.p; a.cf_val = vals<T>(c.Cf);
  }
  a.x = x;
  a.y = y;
  a.fluid_only = fluid_only ? 1 : 0;
  a.gU = solid_only ? 0u : (unsigned)((c.N2 + kRowsPerBlock - 1) / kRowsPerBlock);
  a.gP = solid_only ? 0u : (unsigned)((c.Np + kRowsPerBlock - 1) / kRowsPerBlock);
  unsigned gS = fluid_only ? 0u : (unsigned)((c.Ns + kRowsPerBlock - 1) / kRowsPerBlock);
  hipLaunchKernelGGL((k_operator<T, Tx, Ty>), dim3(a.gU + a.gP + gS), dim3(kOpBlock), 0, c.stream, a);
  FSI_CHECK_LAUNCH();
}

// Fluid rows matrix-free (structured-grid products enabled, FP64): one tiled launch for
// the velocity and pressure rows, then the solid row group of the fused kernel.
static void fluid_rows_stencil(Ctx &c, const double *x, double *y, bool fluid_only) {
  const bool cft = !fluid_only && c.CfT.rowptr.p != nullptr;
  const double *xl = x + 2 * c.N2 + c.Np + 2 * c.Ns;
  stencil_fluid_rows<double>(c.n, (const StencilTable<double> *)c.mgu.lv[0].stab64.p,
                             (const DivTable<double> *)c.divtab64.p, x, y, cft ? c.CfT.rowptr.p : nullptr,
                             cft ? c.CfT.col.p : nullptr, cft ? c.CfT.val.p : nullptr, cft ? xl : nullptr,
                             c.Ns, c.stream);
}

template <typename T, typename Tx>
void apply_operator(Ctx &c, const Tx *x, double *y, bool fluid_only) {
  if constexpr (std::is_same<T, double>::value && std::is_same<Tx, double>::value) {
    if (c.mgu.stencil) {
      fluid_rows_stencil(c, x, y, fluid_only);
      if (!fluid_only) launch_operator<double, double, double>(c, x, y, false, true);
      return;
    }
  }
  launch_operator<T, Tx, double>(c, x, y, fluid_only);
}
template void apply_operator<double, double>(Ctx &, const double *, double *, bool);
template void apply_operator<float, double>(Ctx &, const double *, double *, bool);

// A11 on [u | p] in one precision (inner solves)
template <typename T>
void apply_a11(Ctx &c, const T *x, T *y) {
  launch_operator<T, T, T>(c, x, y, true);
}
template void apply_a11<double>(Ctx &, const double *, double *);
template void apply_a11<float>(Ctx &, const float *, float *);

// A11 on FP64 vectors, arithmetic and matrix values in TA (FP32: values from the shadows).
// FP64 with the structured-grid products enabled: one matrix-free tiled launch
// (A_f stencil, B and B^T from their class tables); otherwise the assembled blocks.
template <typename TA>
void apply_a11_on64(Ctx &c, const double *x, double *y) {
  if constexpr (std::is_same<TA, double>::value) {
    if (c.mgu.stencil) {
      fluid_rows_stencil(c, x, y, true);
      return;
    }
  }
  launch_operator<TA, double, double>(c, x, y, true);
}
template void apply_a11_on64<double>(Ctx &, const double *, double *);
template void apply_a11_on64<float>(Ctx &, const double *, double *);

// ---- right-hand side of eq. (matrix)
__global__ void k_rhs_u(int64_t N2, const int *rp, const int *col, const double *M,
                        const unsigned char *bnd, const double *u, double rdt, double *b) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t r = gid / kG;
  int lane = (int)(gid % kG);
  if (r >= N2) return;
  double sx = 0, sy = 0;
  for (int k = rp[r] + lane; k < rp[r + 1]; k += kG) {
    int j = col[k];
    if (bnd[j]) continue;
    sx += M[k] * u[j];
    sy += M[k] * u[N2 + j];
  }
  sx = group_sum<kG>(sx);
  sy = group_sum<kG>(sy);
  if (lane == 0) {
    b[r] = bnd[r] ? 0.0 : rdt * sx;
    b[N2 + r] = bnd[r] ? 0.0 : rdt * sy;
  }
}

__global__ void k_rhs_s(int64_t Ns, const int *rp, const int *col, const double *Cs, const double *X,
                        double minv_dt, double *bX) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t l = gid / kG;
  int lane = (int)(gid % kG);
  if (l >= Ns) return;
  double sx = 0, sy = 0;
  for (int k = rp[l] + lane; k < rp[l + 1]; k += kG) {
    int j = col[k];
    sx += Cs[k] * X[j];
    sy += Cs[k] * X[Ns + j];
  }
  sx = group_sum<kG>(sx);
  sy = group_sum<kG>(sy);
  if (lane == 0) {
    bX[l] = 0.0;
    bX[Ns + l] = 0.0;
    bX[2 * Ns + l] = minv_dt * sx;
    bX[3 * Ns + l] = minv_dt * sy;
  }
}

void build_rhs(Ctx &c, const double *u_n, const double *X_n, double *b) {
  hipStream_t s = c.stream;
  hipLaunchKernelGGL(k_rhs_u, dim3(grid_for(c.N2 * kG, 256)), dim3(256), 0, s, c.N2, c.Af.rowptr.p,
                     c.Af.col.p, c.Mf.p, c.bnd.p, u_n, c.rho / c.dt, b);
  fill(b + 2 * c.N2, c.Np, 0.0, s);
  hipLaunchKernelGGL(k_rhs_s, dim3(grid_for(c.Ns * kG, 256)), dim3(256), 0, s, c.Ns, c.S.rowptr.p,
                     c.S.col.p, c.Cs.p, X_n, -1.0 / c.dt, b + 2 * c.N2 + c.Np);
  FSI_CHECK_LAUNCH();
}

}  // namespace fsi
