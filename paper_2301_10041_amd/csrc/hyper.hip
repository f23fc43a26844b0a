// The nonlinear solid on the device: the exponential law of the paper's nonlinear test
// (Sec. 6.2), W(F) = (gamma / (2 eta)) exp(eta (tr F^T F - 2)), its stress
// P(F) = dW/dF = gamma e F with e = exp(eta (|F|^2 - 2)), and the tangent
// dP_ab/dF_cd = gamma e (delta_ac delta_bd + 2 eta F_ab F_cd); eta = 0 is the linear law P = gamma F.
//
// On P1 triangles F is constant per triangle E; with G_i the gradient of the basis function of
// local vertex i,
//   R(X)_{l,a} = sum_{E ∋ l} |E| P_ab(F_E) G_{l,b}                      (solid residual)
//   K(X)_{(l,a),(j,c)} = sum_{E ∋ l, j} |E| gamma e_E [ (G_l . G_j) delta_ac
//                                                 + 2 eta (F_E G_l)_a (F_E G_j)_c ]   (tangent)
// K is stored as 2 x 2 blocks (xx, xy, yx, yy) on the solid P1 pattern.  One thread per solid
// node gathers the triangles around it (sorted by element), so every sum has a fixed order.
//
// Newton's method for one step (Sec. 4, last paragraph; Sec. 6: stop on a 1e-6 reduction of
// the Euclidean norm of the relative residual): the residual of eq. (matrix) with A_s X
// replaced by R(X), the Jacobian systems solved by the flexible GMRES of solve.hip with the
// tangent in place of A_s (operator and block preconditioners).
#include <chrono>
#include <cmath>

#include "ctx.h"
#include "kernels.h"

namespace fsi {

__global__ void k_solid_law(int64_t ns, const int *__restrict__ n2e_ptr, const int *__restrict__ n2e,
                            const int *__restrict__ tri, const double *__restrict__ xy,
                            const int *__restrict__ rowptr, const int *__restrict__ col,
                            const double *__restrict__ X, double gamma, double eta, double *R, double *Kt) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ns) return;
  const int r0 = rowptr[l], r1 = rowptr[l + 1];
  if (Kt)
    for (int k = 4 * r0; k < 4 * r1; ++k) Kt[k] = 0.0;
  double rx = 0.0, ry = 0.0;
  for (int q = n2e_ptr[l]; q < n2e_ptr[l + 1]; ++q) {
    const int e = n2e[q] >> 2, a = n2e[q] & 3;
    const int v[3] = {tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]};
    double x[3], y[3];
    for (int m = 0; m < 3; ++m) { x[m] = xy[v[m]]; y[m] = xy[ns + v[m]]; }
    const double d = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    const double area = 0.5 * d;
    const double gx[3] = {(y[1] - y[2]) / d, (y[2] - y[0]) / d, (y[0] - y[1]) / d};
    const double gy[3] = {(x[2] - x[1]) / d, (x[0] - x[2]) / d, (x[1] - x[0]) / d};
    // F_E = sum_m X_m G_m^T
    double f00 = 0.0, f01 = 0.0, f10 = 0.0, f11 = 0.0;
    for (int m = 0; m < 3; ++m) {
      const double Xx = X[v[m]], Xy = X[ns + v[m]];
      f00 += Xx * gx[m]; f01 += Xx * gy[m];
      f10 += Xy * gx[m]; f11 += Xy * gy[m];
    }
    const double ge = gamma * exp(eta * (f00 * f00 + f01 * f01 + f10 * f10 + f11 * f11 - 2.0));
    // P G_a
    rx += area * ge * (f00 * gx[a] + f01 * gy[a]);
    ry += area * ge * (f10 * gx[a] + f11 * gy[a]);
    if (Kt) {
      const double ax = f00 * gx[a] + f01 * gy[a], ay = f10 * gx[a] + f11 * gy[a];   // F G_a
      const double w = area * ge, w2 = 2.0 * eta * area * ge;
      for (int b = 0; b < 3; ++b) {
        int pos = r0;
        while (pos < r1 && col[pos] != v[b]) ++pos;
        const double bx = f00 * gx[b] + f01 * gy[b], by = f10 * gx[b] + f11 * gy[b];   // F G_b
        const double gg = gx[a] * gx[b] + gy[a] * gy[b];
        Kt[4 * pos] += w * gg + w2 * ax * bx;
        Kt[4 * pos + 1] += w2 * ax * by;
        Kt[4 * pos + 2] += w2 * ay * bx;
        Kt[4 * pos + 3] += w * gg + w2 * ay * by;
      }
    }
  }
  if (R) {
    R[l] = rx;
    R[ns + l] = ry;
  }
}

// The solid rows of the nonlinear residual: y_X = R(X) - C_s lam (both components).
__global__ void k_solid_rows_nl(int64_t ns, const int *__restrict__ rowptr, const int *__restrict__ col,
                                const double *__restrict__ Cs, const double *__restrict__ lam,
                                const double *__restrict__ R, double *yX) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ns) return;
  double sx = 0.0, sy = 0.0;
  for (int k = rowptr[l]; k < rowptr[l + 1]; ++k) {
    const int j = col[k];
    sx += Cs[k] * lam[j];
    sy += Cs[k] * lam[ns + j];
  }
  yX[l] = R[l] - sx;
  yX[ns + l] = R[ns + l] - sy;
}

static void law_params(const Ctx &c, double &gamma, double &eta) {
  if (c.law == FSI_LAW_EXP) {
    gamma = c.law_gamma;
    eta = c.law_eta;
  } else {   // the linear law kappa F
    gamma = c.kappa;
    eta = 0.0;
  }
}

// R(X) into R (2 Ns, may be null) and, with tangent, K(X) into the context (c.Kt and its FP32
// copy).  X: device [x | y] (2 Ns).
void solid_law(Ctx &c, const double *X, double *R, bool tangent) {
  const int64_t ns = c.Ns;
  double gamma, eta;
  law_params(c, gamma, eta);
  if (tangent) {
    c.Kt.reserve(4 * (size_t)c.S.nnz);
    c.Kt32.reserve(4 * (size_t)c.S.nnz);
  }
  hipLaunchKernelGGL(k_solid_law, dim3(grid_for(ns, 128)), dim3(128), 0, c.stream, ns, c.n2e_ptr.p, c.n2e.p,
                     c.tri.p, c.ref_xy.p, c.S.rowptr.p, c.S.col.p, X, gamma, eta, R, tangent ? c.Kt.p : nullptr);
  FSI_CHECK_LAUNCH();
  if (tangent) {
    convert(c.Kt32.p, c.Kt.p, 4 * c.S.nnz, c.stream);
    c.use_kt = true;
  }
}

template <typename T, typename Tx>
void apply_operator(Ctx &c, const Tx *x, double *y, bool fluid_only);
void gmres_solve(Ctx &c, const fsi_solve_opts &o, const double *b, double *x, fsi_solve_stats *st);

// y = G(x): eq. (matrix) with the solid product replaced by R(X) (R computed into c.nl_R).
static void nonlinear_apply(Ctx &c, const double *x, double *y) {
  const int64_t ns = c.Ns, off = 2 * c.N2 + c.Np;
  const bool kt = c.use_kt;
  c.use_kt = false;   // the operator's other rows do not depend on the solid block
  apply_operator<double, double>(c, x, y, false);
  c.use_kt = kt;
  solid_law(c, x + off, c.nl_R.p, false);
  hipLaunchKernelGGL(k_solid_rows_nl, dim3(grid_for(ns, 256)), dim3(256), 0, c.stream, ns, c.S.rowptr.p,
                     c.S.col.p, c.Cs.p, x + off + 2 * ns, c.nl_R.p, y + off);
  FSI_CHECK_LAUNCH();
}

__global__ void k_sub(double *r, const double *b, const double *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - y[i];
}

__global__ void k_add(double *x, const double *d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}

// ||v||_2 on the host (FP64, fixed partition: the reduction kernels of kernels.h); synchronises
static double norm2(Ctx &c, const double *v, int64_t n) {
  c.dscal.reserve(512);
  multidot(v, 0, 1, v, n, c.dscal.p, c.red, c.stream);
  FSI_HIP(hipMemcpyAsync(c.hpin, c.dscal.p, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  FSI_HIP(hipStreamSynchronize(c.stream));
  return std::sqrt(c.hpin[0]);
}

void newton_step(Ctx &c, const fsi_solve_opts &o, const fsi_newton_opts &no, const double *u_n, const double *X_n,
                 const double *f_X, double *x, fsi_newton_stats *st) {
  using clk = std::chrono::steady_clock;
  FSI_REQUIRE(no.rtol > 0.0 && no.maxit >= 1, FSI_E_ARG, "Newton needs rtol > 0 and maxit >= 1");
  const int64_t N = c.N, ns = c.Ns, off = 2 * c.N2 + c.Np;
  fsi_newton_stats s{};
  const bool kt0 = c.use_kt;
  auto t0 = clk::now();
  assemble_coupling(c, X_n, true);
  FSI_HIP(hipStreamSynchronize(c.stream));
  auto t1 = clk::now();
  s.t_coup = std::chrono::duration<double>(t1 - t0).count();
  c.nl_b.reserve(N);
  c.nl_r.reserve(N);
  c.nl_d.reserve(N);
  c.nl_R.reserve(2 * ns);
  double *b = c.nl_b.p, *r = c.nl_r.p, *d = c.nl_d.p;
  build_rhs(c, u_n, X_n, b);
  if (f_X) hipLaunchKernelGGL(k_add, dim3(vgrid(2 * ns)), dim3(256), 0, c.stream, b + off, f_X, 2 * ns);
  FSI_CHECK_LAUNCH();
  double res0 = 0.0, res = 0.0;
  int k = 0;
  bool conv = false;
  try {
    for (k = 0;; ++k) {
      auto ta = clk::now();
      c.use_kt = false;
      nonlinear_apply(c, x, d);
      hipLaunchKernelGGL(k_sub, dim3(vgrid(N)), dim3(256), 0, c.stream, r, b, d, N);
      FSI_CHECK_LAUNCH();
      res = norm2(c, r, N);
      FSI_REQUIRE(std::isfinite(res), FSI_E_NONFINITE, "non-finite Newton residual");
      if (k == 0) res0 = res;
      s.t_res += std::chrono::duration<double>(clk::now() - ta).count();
      if (res == 0.0 || res <= no.rtol * res0) {
        conv = true;
        break;
      }
      if (k == no.maxit) break;
      // the Jacobian system J(x_k) d = r with the tangent K(X_k) in place of A_s
      auto tb = clk::now();
      solid_law(c, x + off, nullptr, true);
      fill(d, N, 0.0, c.stream);
      fsi_solve_stats ls{};
      gmres_solve(c, o, r, d, &ls);
      hipLaunchKernelGGL(k_add, dim3(vgrid(N)), dim3(256), 0, c.stream, x, d, N);
      FSI_CHECK_LAUNCH();
      FSI_HIP(hipStreamSynchronize(c.stream));
      s.t_solve += std::chrono::duration<double>(clk::now() - tb).count();
      s.its_total += ls.its;
      s.inner_its += ls.inner_its;
    }
  } catch (...) {
    c.use_kt = kt0;
    throw;
  }
  c.use_kt = kt0;
  s.nit = k;
  s.converged = conv ? 1 : 0;
  s.res0 = res0;
  s.res = res;
  if (st) *st = s;
  if (!conv) throw Error(FSI_E_NOCONV, "Newton did not reach its tolerance in maxit iterations");
}

}  // namespace fsi
