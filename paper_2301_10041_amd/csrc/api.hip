#include <algorithm>
// extern "C" entry points of libfsi (declared in include/fsi.h).  Every call catches
// the library's exceptions and returns an fsi_status; the message is kept in the context.
#include <chrono>
#include <cmath>
#include <cstring>

#include "ctx.h"
#include "q2.h"
#include "lattice.h"
#include "stencil.h"
#include "kernels.h"

struct fsi_ctx {
  fsi::Ctx c;
};

namespace fsi {

Ctx::~Ctx() {
  drop_graphs();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (aux_stream) (void)hipStreamDestroy(aux_stream);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  for (hipEvent_t e : ev_ms)
    if (e) (void)hipEventDestroy(e);
  if (hpin) (void)hipHostFree(hpin);
  if (bat_h) (void)hipHostFree(bat_h);
  if (gi_h) (void)hipHostFree(gi_h);
}

void Prof::begin(hipStream_t s) {
  if (used + 2 > ev.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      FSI_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
  }
  FSI_HIP(hipEventRecord(ev[used], s));
}

void Prof::end(hipStream_t s) {
  FSI_HIP(hipEventRecord(ev[used + 1], s));
  used += 2;
}

double Prof::total_ms(int64_t &launches) {
  double t = 0.0;
  for (size_t k = 0; k + 1 < used; k += 2) {
    float ms = 0.f;
    FSI_HIP(hipEventSynchronize(ev[k + 1]));
    FSI_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
    t += ms;
  }
  launches = (int64_t)(used / 2);
  return t;
}

Prof::~Prof() {
  for (auto e : ev) (void)hipEventDestroy(e);
}

size_t Ctx::device_bytes() const {
  size_t b = Af.bytes() + Mf.bytes() + B.bytes() + BT.bytes() + Mp.bytes() + Mp_dinv.bytes() +
             Mp_dinv32.bytes() + bnd.bytes();
  b += tri.bytes() + ref_xy.bytes() + ref_area.bytes() + n2e_ptr.bytes() + n2e.bytes() + S.bytes() +
       Cs.bytes() + Cs32.bytes() + Cs_dinv.bytes() + Cs_dinv32.bytes() + s_ecol.bytes() + s_eas.bytes() +
       s_ecs.bytes();
  b += Cf.bytes() + CfT.bytes() + cand_off.bytes() + piece_cnt.bytes() + pair_E.bytes() +
       pair_T.bytes() + piece_L.bytes() + e_piece.bytes() + cft_fill.bytes() + dflag.bytes() +
       cft_tcol.bytes() + cft_tval.bytes() + cft_long.bytes() + scan_tmp.bytes() + cf_defer.bytes() + cf_defer2.bytes() + cf_huge.bytes() + cf_wflag.bytes() + cf_wval.bytes();
  b += inc_box.bytes() + inc_moved.bytes() + inc_prevT.bytes() + inc_X.bytes() + inc_flag.bytes() + cft_tsrc.bytes() +
       cft_perm.bytes();
  b += mgu.bytes() + mgp.bytes();
  for (int i = 0; i < 9; ++i) b += inner.v64[i].bytes() + inner.v32[i].bytes();
  b += outer.V.bytes() + outer.Z.bytes() + outer.w.bytes() + outer.r.bytes() + outer.x32.bytes() +
       outer.y32.bytes();
  b += red.bytes() + dscal.bytes() + tmpN.bytes() + tmpS.bytes();
  b += ms_state.bytes() + ms_red.bytes() + ms_x.bytes() + ms_part.bytes() + ms_dot.bytes() + ms_vh.bytes() +
       ms_hist.bytes() + ms_coef.bytes() + gi_V.bytes() + gi_Z.bytes() + gi_part.bytes() + gi_dh.bytes() +
       gi_sc.bytes() + pc_in.bytes() +
       pc_out.bytes();
  return b;
}

// Footprint estimate made before any allocation (FP64 + FP32 shadows, MG with the dense
// coarsest inverses, Krylov with m = 30 and both precisions' inner vectors).
static size_t estimate_bytes(int64_t n, int64_t ns, int64_t nt) {
  double n2 = (double)n * n;
  double zaf = 46 * n2, zb = 19 * n2, N2 = 4 * n2, Np = n2, N = 2 * N2 + Np + 4 * ns;
  double fluid = zaf * (32 + 4 + 8 + 16) + 2 * zb * (16 + 4 + 8) + 9 * Np * 12 + 4 * (N2 + Np);
  double mg = fluid * 0.45 + 10 * N2 * 12 / 3;
  double krylov = 61 * N * 8 + 9 * (2 * N2 + Np) * 12 + 4 * N * 8 +
                  std::min(32 * (2 * N2 + Np) * 8, (double)(2ll << 30));   // MINRES Lanczos block
  // the dense inverses of the coarsest velocity and pressure levels (FP64 + FP32)
  const std::vector<int> lc = mg_level_cells((int)n);
  const int cu = lc[mg_velocity_levels(lc) - 1], cp = lc.back();
  const double mu = 2.0 * (2 * cu + 1) * (2 * cu + 1), mp = (double)(cp + 1) * (cp + 1);
  mg += (mu * mu + mp * mp) * 12;
  double solid = ns * (7 * 12 * 2 + 200 + 8 * 20) + nt * 60 + 60 * ns * 12;
  double cf = nt * 12 * (18 * 8 + 16) + 2 * 60 * ns * 12 + N2 * 8;
  // fixed work space (reduction partials, device scalars, pinned staging, small
  // buffers) and a 10% margin so that the estimate bounds the measured footprint
  return (size_t)(1.1 * (fluid + mg + krylov + solid + cf) + (4 << 20));
}

}  // namespace fsi

using fsi::Ctx;
using fsi::Error;

static thread_local std::string g_create_error;

template <typename F>
static int guarded(fsi_ctx *h, F &&f) {
  try {
    f();
    return FSI_OK;
  } catch (const Error &e) {
    if (h) h->c.last_error = e.what();
    else g_create_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    if (h) h->c.last_error = "host allocation failed";
    return FSI_E_NOMEM;
  } catch (const std::exception &e) {
    if (h) h->c.last_error = e.what();
    return FSI_E_HIP;
  }
}

extern "C" {

static int create_ctx(const fsi_fluid_desc *fluid, const fsi_solid_desc *solid, void *hip_stream, size_t hbm_budget,
                      fsi_ctx **out, int pair) {
  if (!out) return FSI_E_ARG;
  *out = nullptr;
  fsi_ctx *h = nullptr;
  int rc = guarded(nullptr, [&] {
    FSI_REQUIRE(fluid && solid, FSI_E_ARG, "null descriptor");
    FSI_REQUIRE(fluid->n >= 2 && fluid->n <= 4096, FSI_E_ARG, "fluid n must be in [2, 4096]");
    FSI_REQUIRE(fluid->nu > 0 && fluid->rho > 0 && fluid->dt > 0, FSI_E_ARG, "nu, rho, dt must be > 0");
    FSI_REQUIRE(solid->n_nodes >= 3 && solid->n_tris >= 1 && solid->xy && solid->tri, FSI_E_ARG,
                "solid mesh needs >= 3 nodes, >= 1 triangle and non-null arrays");
    FSI_REQUIRE(solid->kappa >= 0, FSI_E_ARG, "kappa must be >= 0");
    const int64_t n = fluid->n, ns = solid->n_nodes, nt = solid->n_tris;
    const bool quads = pair == FSI_PAIR_Q2P1DISC;
    FSI_REQUIRE(!quads || ns >= 4, FSI_E_ARG, "a quadrilateral mesh needs >= 4 nodes");
    if (hbm_budget && !quads) {
      size_t est = fsi::estimate_bytes(n, ns, nt);
      FSI_REQUIRE(est <= hbm_budget, FSI_E_NOMEM,
                  "estimated footprint " + std::to_string(est) + " B exceeds the budget");
    }
    h = new fsi_ctx();
    Ctx &c = h->c;
    c.pair = pair;
    c.n = fluid->n;
    c.nu = fluid->nu;
    c.rho = fluid->rho;
    c.dt = fluid->dt;
    c.kappa = solid->kappa;
    c.N2 = (2 * n + 1) * (2 * n + 1);
    c.Np = quads ? 3 * n * n : (n + 1) * (n + 1);
    c.Ns = ns;
    c.Nt = nt;
    c.N = 2 * c.N2 + c.Np + 4 * ns;
    c.stream = (hipStream_t)hip_stream;
    c.budget = hbm_budget;
    FSI_HIP(hipGetDevice(&c.device));
    fsi::coupling_scratch_init(c.device);
    c.h_tri.assign(solid->tri, solid->tri + (quads ? 4 : 3) * nt);
    c.h_xy.assign(solid->xy, solid->xy + 2 * ns);
    FSI_HIP(hipHostMalloc((void **)&c.hpin, 4096 * sizeof(double), hipHostMallocDefault));
    FSI_HIP(hipStreamCreateWithFlags(&c.aux_stream, hipStreamNonBlocking));
    FSI_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
    FSI_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
    for (hipEvent_t &e : c.ev_ms) FSI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    fsi::build_solid(c);
    if (quads) {   // the assembled operators only: the matrix-free kernels are the triangle pair's
      fsi::build_fluid_q2(c);
      fsi::build_multigrid_q2(c);
    } else {
      fsi::build_fluid(c);
      fsi::build_multigrid(c);
      c.mgu.stencil = c.mgp.stencil = true;
    }
    // graphs keep the preconditioner on one stream (the pressure chain no longer beside the
    // velocity cycle) and check convergence every second MINRES step: with the coarse ends of
    // both cycles in one launch each they measured slower than the two streams at every size
    // (32^2 27.1 / 23.3 ms, 128^2 54.6 / 43.8 ms per FP64 step, batches of 8 likewise), so
    // they are off unless fsi_set_graphs asks for them
    c.use_graphs = false;
    fsi::make_shadow(c.Af, c.stream);
    fsi::make_shadow(c.B, c.stream);
    fsi::make_shadow(c.BT, c.stream);
    fsi::make_shadow(c.S, c.stream);
    c.tmpN.reserve(c.N);
    c.tmpS.reserve(12 * ns);
    fsi::reserve_coupling(c);
    c.dscal.alloc(512);
    FSI_HIP(hipStreamSynchronize(c.stream));
    if (hbm_budget)
      FSI_REQUIRE(c.device_bytes() <= hbm_budget, FSI_E_NOMEM, "device footprint exceeds the budget");
  });
  if (rc != FSI_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return FSI_OK;
}

int fsi_create(const fsi_fluid_desc *fluid, const fsi_solid_desc *solid, void *hip_stream,
               size_t hbm_budget, fsi_ctx **out) {
  return create_ctx(fluid, solid, hip_stream, hbm_budget, out, FSI_PAIR_P2P1);
}

int fsi_create_q2(const fsi_fluid_desc *fluid, const fsi_solid_desc *solid, void *hip_stream, size_t hbm_budget,
                  fsi_ctx **out) {
  return create_ctx(fluid, solid, hip_stream, hbm_budget, out, FSI_PAIR_Q2P1DISC);
}

void fsi_destroy(fsi_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->c.stream);
  delete ctx;
}

int fsi_set_solid(fsi_ctx *ctx, const fsi_solid_desc *solid) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1, FSI_E_STATE, "fsi_set_solid takes the triangle pair only");
    FSI_REQUIRE(solid && solid->n_nodes >= 3 && solid->n_tris >= 1 && solid->xy && solid->tri,
                FSI_E_ARG, "solid mesh needs >= 3 nodes, >= 1 triangle and non-null arrays");
    FSI_REQUIRE(solid->kappa >= 0, FSI_E_ARG, "kappa must be >= 0");
    Ctx &c = ctx->c;
    FSI_HIP(hipStreamSynchronize(c.stream));
    const int64_t ns = solid->n_nodes, nt = solid->n_tris;
    c.have_cf = false;
    c.inc_valid = false;
    c.kappa = solid->kappa;
    c.Ns = ns;
    c.Nt = nt;
    c.N = 2 * c.N2 + c.Np + 4 * ns;
    c.h_tri.assign(solid->tri, solid->tri + 3 * nt);
    c.h_xy.assign(solid->xy, solid->xy + 2 * ns);
    c.use_kt = false;   // a tangent of the previous solid no longer fits its pattern
    c.Kt.release();
    fsi::build_solid(c);
    fsi::make_shadow(c.S, c.stream);
    c.tmpN.reserve(c.N);
    c.tmpS.reserve(12 * ns);
    fsi::reserve_coupling(c);
    FSI_HIP(hipStreamSynchronize(c.stream));
  });
}

int fsi_set_smoother(fsi_ctx *ctx, int kind) {
  if (!ctx) return FSI_E_ARG;
  if (kind != FSI_SMOOTH_CSR && kind != FSI_SMOOTH_STENCIL) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1 || kind == FSI_SMOOTH_CSR, FSI_E_STATE,
                "the matrix-free smoother takes the triangle pair only");
    FSI_HIP(hipStreamSynchronize(ctx->c.stream));   // captured graphs may still be running
    ctx->c.drop_graphs();
    ctx->c.mgu.stencil = ctx->c.mgp.stencil = kind == FSI_SMOOTH_STENCIL;
  });
}

int fsi_set_inner_check(fsi_ctx *ctx, int mode) {
  if (!ctx) return FSI_E_ARG;
  if (mode != FSI_CHECK_AUTO && mode != FSI_CHECK_EVERY_STEP && mode != FSI_CHECK_LAGGED) return FSI_E_ARG;
  ctx->c.ms_check = mode;
  return FSI_OK;
}

int fsi_set_graphs(fsi_ctx *ctx, int enable) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_HIP(hipStreamSynchronize(ctx->c.stream));   // captured graphs may still be running
    ctx->c.drop_graphs();
    ctx->c.use_graphs = enable != 0;
  });
}

int fsi_footprint(const fsi_fluid_desc *fluid, int64_t n_nodes, int64_t n_tris, size_t *bytes) {
  if (!fluid || !bytes || fluid->n < 2 || n_nodes < 3 || n_tris < 1) return FSI_E_ARG;
  *bytes = fsi::estimate_bytes(fluid->n, n_nodes, n_tris);
  return FSI_OK;
}

int fsi_set_stream(fsi_ctx *ctx, void *hip_stream) {
  if (!ctx) return FSI_E_ARG;
  ctx->c.stream = (hipStream_t)hip_stream;
  return FSI_OK;
}

int fsi_sizes(const fsi_ctx *ctx, fsi_sizes_t *o) {
  if (!ctx || !o) return FSI_E_ARG;
  const Ctx &c = ctx->c;
  std::memset(o, 0, sizeof(*o));
  o->N2 = c.N2; o->Np = c.Np; o->Ns = c.Ns; o->Nt = c.Nt; o->N = c.N;
  o->off_ux = 0; o->off_uy = c.N2; o->off_p = 2 * c.N2; o->off_Xx = 2 * c.N2 + c.Np;
  o->off_Xy = o->off_Xx + c.Ns; o->off_lx = o->off_Xy + c.Ns; o->off_ly = o->off_lx + c.Ns;
  o->nnz_Af = c.Af.nnz; o->nnz_B = c.B.nnz; o->nnz_s = c.S.nnz;
  o->nnz_Cf = c.have_cf ? c.Cf.nnz : 0;
  o->n_pairs = c.have_cf ? c.n_pairs : 0;
  o->device_bytes = (int64_t)c.device_bytes();
  o->mg_levels_u = (int32_t)c.mgu.lv.size();
  o->mg_levels_p = (int32_t)c.mgp.lv.size();
  return FSI_OK;
}

int fsi_assemble_coupling(fsi_ctx *ctx, const double *Xn, fsi_coupling_info *info) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(Xn, FSI_E_ARG, "null X^n");
    fsi::assemble_coupling(ctx->c, Xn, info != nullptr);
    if (info) {
      FSI_HIP(hipStreamSynchronize(ctx->c.stream));
      info->n_pairs = ctx->c.n_pairs;
      info->nnz = ctx->c.Cf.nnz;
    }
  });
}

int fsi_set_coupling_mode(fsi_ctx *ctx, int mode) {
  if (!ctx) return FSI_E_ARG;
  if (mode != FSI_COUPLING_FULL && mode != FSI_COUPLING_INCREMENTAL) return FSI_E_ARG;
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    FSI_REQUIRE(c.pair == FSI_PAIR_P2P1 || mode == FSI_COUPLING_FULL, FSI_E_STATE,
                "the time-coherent coupling assembly takes the triangle pair only");
    if (c.cf_mode != mode) c.inc_valid = false;
    c.cf_mode = mode;
  });
}

int fsi_get_coupling_counts(const fsi_ctx *ctx, fsi_coupling_counts *out) {
  if (!ctx || !out) return FSI_E_ARG;
  const Ctx &c = ctx->c;
  out->calls = c.inc_counts[0];
  out->rebuilds = c.inc_counts[1];
  out->pattern_builds = c.inc_counts[2];
  out->value_refills = c.inc_counts[3];
  out->unchanged = c.inc_counts[4];
  return FSI_OK;
}

int fsi_assemble_coupling_noalloc(fsi_ctx *ctx, const double *Xn, fsi_coupling_info *info) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1, FSI_E_STATE, "the allocation-free coupling assembly takes the triangle pair only");
    FSI_REQUIRE(Xn, FSI_E_ARG, "null X^n");
    fsi::assemble_coupling_noalloc(ctx->c, Xn);
    if (info) {
      FSI_HIP(hipStreamSynchronize(ctx->c.stream));
      info->n_pairs = ctx->c.n_pairs;
      info->nnz = ctx->c.Cf.nnz;
    }
  });
}

int fsi_build_rhs(fsi_ctx *ctx, const double *u_n, const double *X_n, double *b) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(u_n && X_n && b, FSI_E_ARG, "null vector");
    fsi::build_rhs(ctx->c, u_n, X_n, b);
  });
}

int fsi_apply_operator(fsi_ctx *ctx, int prec, const double *x, double *y) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(x && y && x != y, FSI_E_ARG, "null or aliased vectors");
    FSI_REQUIRE(ctx->c.have_cf, FSI_E_STATE, "call fsi_assemble_coupling first");
    if (prec == FSI_FP64) fsi::apply_operator<double, double>(ctx->c, x, y, false);
    else if (prec == FSI_FP32) fsi::apply_operator<float, double>(ctx->c, x, y, false);
    else throw Error(FSI_E_ARG, "unknown precision");
  });
}

int fsi_apply_precond(fsi_ctx *ctx, int pc, int prec, const double *r, double *z) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(r && z && r != z, FSI_E_ARG, "null or aliased vectors");
    ctx->c.dscal.reserve(512);
    fsi::apply_precond(ctx->c, pc, prec, r, z);
  });
}

int fsi_set_inner(fsi_ctx *ctx, double inner_rtol, int32_t inner_maxit) {
  if (!ctx) return FSI_E_ARG;
  if (inner_maxit < 0) return FSI_E_ARG;
  ctx->c.inner_rtol = inner_rtol;
  if (inner_maxit > 0) ctx->c.inner_maxit = inner_maxit;
  return FSI_OK;
}

int fsi_set_inner_mode(fsi_ctx *ctx, int32_t mode, int32_t cycles) {
  if (!ctx) return FSI_E_ARG;
  if (mode < FSI_INNER_MINRES || mode > FSI_INNER_GMRES || cycles < 0 || cycles > 100) return FSI_E_ARG;
  if (ctx->c.pair != FSI_PAIR_P2P1 && mode != FSI_INNER_MINRES) {
    ctx->c.last_error = "inner modes other than MINRES take the triangle pair only";
    return FSI_E_STATE;
  }
  ctx->c.inner_mode = mode;
  ctx->c.inner_cycles = cycles > 0 ? cycles : 1;
  return FSI_OK;
}

int fsi_gmres_solve(fsi_ctx *ctx, const fsi_solve_opts *opts, const double *b, double *x,
                    fsi_solve_stats *stats) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(opts && b && x && b != x, FSI_E_ARG, "null options or vectors");
    auto t0 = std::chrono::steady_clock::now();
    fsi_solve_stats st{};
    int rc = FSI_OK;
    try {
      fsi::gmres_solve(ctx->c, *opts, b, x, &st);
    } catch (const Error &e) {
      if (e.code != FSI_E_NOCONV) throw;
      rc = e.code;
      ctx->c.last_error = e.what();
    }
    FSI_HIP(hipStreamSynchronize(ctx->c.stream));
    st.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    if (rc != FSI_OK) throw Error(rc, ctx->c.last_error);
  });
}

int fsi_step(fsi_ctx *ctx, const fsi_solve_opts *opts, const double *u_n, const double *X_n,
             double *state, fsi_solve_stats *stats) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(opts && u_n && X_n && state, FSI_E_ARG, "null options or vectors");
    Ctx &c = ctx->c;
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    fsi::assemble_coupling(c, X_n, true);
    FSI_HIP(hipStreamSynchronize(c.stream));
    auto t1 = clk::now();
    double *b = c.tmpN.p;
    fsi::build_rhs(c, u_n, X_n, b);
    fsi::fill(state, c.N, 0.0, c.stream);
    FSI_HIP(hipStreamSynchronize(c.stream));
    auto t2 = clk::now();
    fsi_solve_stats st{};
    int rc = FSI_OK;
    try {
      fsi::gmres_solve(c, *opts, b, state, &st);
    } catch (const Error &e) {
      if (e.code != FSI_E_NOCONV) throw;
      rc = e.code;
      c.last_error = e.what();
    }
    FSI_HIP(hipStreamSynchronize(c.stream));
    auto t3 = clk::now();
    st.t_coup = std::chrono::duration<double>(t1 - t0).count();
    st.t_rhs = std::chrono::duration<double>(t2 - t1).count();
    st.t_solve = std::chrono::duration<double>(t3 - t2).count();
    if (stats) *stats = st;
    if (rc != FSI_OK) throw Error(rc, c.last_error);
  });
}

int fsi_step_batch(int32_t K, fsi_ctx *const *ctxs, const fsi_solve_opts *opts, const double *const *u_n,
                   const double *const *X_n, double *const *state, fsi_solve_stats *stats, int32_t *rc) {
  if (K < 1 || K > FSI_MAX_LANES || !ctxs || !ctxs[0]) return FSI_E_ARG;
  fsi_ctx *lead = ctxs[0];
  return guarded(lead, [&] {
    FSI_REQUIRE(opts && u_n && X_n && state, FSI_E_ARG, "null options or arrays");
    std::vector<Ctx *> cs(K);
    for (int k = 0; k < K; ++k) {
      FSI_REQUIRE(ctxs[k] && u_n[k] && X_n[k] && state[k], FSI_E_ARG, "null context or vector in the batch");
      cs[k] = &ctxs[k]->c;
      FSI_REQUIRE(cs[k]->pair == FSI_PAIR_P2P1, FSI_E_STATE, "fsi_step_batch takes the triangle pair only");
      for (int q = 0; q < k; ++q) FSI_REQUIRE(cs[q] != cs[k], FSI_E_ARG, "a context appears twice in the batch");
      const Ctx &a = *cs[0], &b = *cs[k];
      FSI_REQUIRE(a.n == b.n && a.nu == b.nu && a.rho == b.rho && a.dt == b.dt, FSI_E_ARG,
                  "systems of a batch need the same fluid grid and parameters");
    }
    hipStream_t s = cs[0]->stream;
    // every context on the leading stream for the call (their own streams drained first)
    struct Streams {
      std::vector<Ctx *> &cs;
      std::vector<hipStream_t> old;
      ~Streams() {
        for (size_t k = 0; k < cs.size(); ++k) cs[k]->stream = old[k];
      }
    } streams{cs, {}};
    for (Ctx *c : cs) {
      streams.old.push_back(c->stream);
      if (c->stream != s) FSI_HIP(hipStreamSynchronize(c->stream));
    }
    for (Ctx *c : cs) c->stream = s;
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    for (int k = 0; k < K; ++k) fsi::assemble_coupling(*cs[k], X_n[k], true);
    FSI_HIP(hipStreamSynchronize(s));
    auto t1 = clk::now();
    std::vector<const double *> b(K);
    for (int k = 0; k < K; ++k) {
      b[k] = cs[k]->tmpN.p;
      fsi::build_rhs(*cs[k], u_n[k], X_n[k], cs[k]->tmpN.p);
      fsi::fill(state[k], cs[k]->N, 0.0, s);
    }
    FSI_HIP(hipStreamSynchronize(s));
    auto t2 = clk::now();
    std::vector<fsi_solve_stats> st(K);
    std::vector<int> rcs(K, FSI_OK);
    fsi::gmres_solve_lanes(cs.data(), K, *opts, b.data(), state, st.data(), rcs.data());
    FSI_HIP(hipStreamSynchronize(s));
    auto t3 = clk::now();
    int first = -1;
    for (int k = 0; k < K; ++k) {
      st[k].t_coup = std::chrono::duration<double>(t1 - t0).count();
      st[k].t_rhs = std::chrono::duration<double>(t2 - t1).count();
      st[k].t_solve = std::chrono::duration<double>(t3 - t2).count();
      if (stats) stats[k] = st[k];
      if (rc) rc[k] = rcs[k];
      if (rcs[k] != FSI_OK && first < 0) first = k;
    }
    if (first >= 0) throw Error(rcs[first], cs[first]->last_error);
  });
}

int fsi_set_law(fsi_ctx *ctx, int law, double gamma, double eta) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(law == FSI_LAW_LINEAR || law == FSI_LAW_EXP, FSI_E_ARG, "unknown solid law");
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1 || law == FSI_LAW_LINEAR, FSI_E_STATE,
                "the nonlinear solid takes the triangle pair only");
    if (law == FSI_LAW_EXP)
      FSI_REQUIRE(gamma > 0.0 && eta >= 0.0 && std::isfinite(gamma) && std::isfinite(eta), FSI_E_ARG,
                  "the exponential law needs gamma > 0 and eta >= 0");
    ctx->c.law = law;
    ctx->c.law_gamma = gamma;
    ctx->c.law_eta = eta;
  });
}

int fsi_solid_residual(fsi_ctx *ctx, const double *X, double *R) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1, FSI_E_STATE, "the nonlinear solid takes the triangle pair only");
    FSI_REQUIRE(X && R && X != R, FSI_E_ARG, "null or aliased vectors");
    fsi::solid_law(ctx->c, X, R, false);
  });
}

int fsi_solid_tangent(fsi_ctx *ctx, const double *X) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1, FSI_E_STATE, "the nonlinear solid takes the triangle pair only");
    if (!X) {
      ctx->c.use_kt = false;
      return;
    }
    fsi::solid_law(ctx->c, X, nullptr, true);
  });
}

int fsi_newton_step(fsi_ctx *ctx, const fsi_solve_opts *opts, const fsi_newton_opts *nopts, const double *u_n,
                    const double *X_n, const double *f_X, double *state, fsi_newton_stats *stats) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    FSI_REQUIRE(ctx->c.pair == FSI_PAIR_P2P1, FSI_E_STATE, "the nonlinear solid takes the triangle pair only");
    FSI_REQUIRE(opts && nopts && u_n && X_n && state, FSI_E_ARG, "null options or vectors");
    fsi_newton_stats st{};
    int rc = FSI_OK;
    try {
      fsi::newton_step(ctx->c, *opts, *nopts, u_n, X_n, f_X, state, &st);
    } catch (const Error &e) {
      if (e.code != FSI_E_NOCONV) throw;
      rc = e.code;
      ctx->c.last_error = e.what();
    }
    FSI_HIP(hipStreamSynchronize(ctx->c.stream));
    if (stats) *stats = st;
    if (rc != FSI_OK) throw Error(rc, ctx->c.last_error);
  });
}

int fsi_export_pairs(fsi_ctx *ctx, int32_t *E, int32_t *T, int64_t cap, int64_t *count) {
  if (!ctx || !count) return FSI_E_ARG;
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    FSI_REQUIRE(c.have_cf, FSI_E_STATE, "call fsi_assemble_coupling first");
    FSI_REQUIRE(c.pairs_kept, FSI_E_STATE,
                "the allocation-free assembly keeps no piece list: call fsi_assemble_coupling");
    *count = c.n_pairs;
    int64_t m = std::min<int64_t>(cap, c.n_pairs);
    if (c.inc_valid) {
      // time-coherent slots: the kept pieces in slot order, which is the canonical order
      std::vector<int32_t> hE(2 * c.n_cand), hT(2 * c.n_cand);
      FSI_HIP(hipMemcpyAsync(hE.data(), c.pair_E.p, hE.size() * 4, hipMemcpyDeviceToHost, c.stream));
      FSI_HIP(hipMemcpyAsync(hT.data(), c.pair_T.p, hT.size() * 4, hipMemcpyDeviceToHost, c.stream));
      FSI_HIP(hipStreamSynchronize(c.stream));
      int64_t k = 0;
      for (size_t q = 0; q < hT.size() && k < m; ++q) {
        if (hT[q] < 0) continue;
        if (E) E[k] = hE[q];
        if (T) T[k] = hT[q];
        ++k;
      }
      return;
    }
    if (m > 0 && E) FSI_HIP(hipMemcpyAsync(E, c.pair_E.p, m * 4, hipMemcpyDeviceToHost, c.stream));
    if (m > 0 && T) FSI_HIP(hipMemcpyAsync(T, c.pair_T.p, m * 4, hipMemcpyDeviceToHost, c.stream));
    FSI_HIP(hipStreamSynchronize(c.stream));
  });
}

int fsi_export_lattice(int32_t n, double nu, double rdt, int32_t table, int32_t *counts, int32_t *offs,
                       double *vals) {
  if (!counts || !offs || !vals) return FSI_E_ARG;
  return guarded(nullptr, [&] {
    FSI_REQUIRE(n >= 2 && n <= 4096, FSI_E_ARG, "n must be in [2, 4096]");
    constexpr int E = FSI_LAT_MAX_ENTRIES;
    std::fill(counts, counts + 9, 0);
    std::fill(offs, offs + 9 * E * 2, 0);
    std::fill(vals, vals + 9 * E * 4, 0.0);
    switch (table) {
      case FSI_LAT_AF: {
        fsi::StencilTable<double> t;
        fsi::StencilTable<float> tf;
        fsi::stencil_tables(n, nu, rdt, t, tf);
        for (int c = 0; c < 4; ++c) {
          counts[c] = t.count[c];
          for (int k = 0; k < t.count[c]; ++k) {
            offs[(c * E + k) * 2] = t.off[c][k][0];
            offs[(c * E + k) * 2 + 1] = t.off[c][k][1];
            for (int q = 0; q < 4; ++q) vals[(c * E + k) * 4 + q] = t.coef[c][k][q];
          }
        }
        break;
      }
      case FSI_LAT_LP:
      case FSI_LAT_MP: {
        fsi::P1Table<double> t;
        fsi::P1Table<float> tf;
        fsi::p1_tables(n, table == FSI_LAT_LP ? fsi::kTableLp : fsi::kTableMp, table == FSI_LAT_LP ? 1 : 0, t, tf);
        static const int nb[fsi::kP1Nbr][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, 1}};
        for (int c = 0; c < 9; ++c) {
          counts[c] = fsi::kP1Nbr;
          for (int k = 0; k < fsi::kP1Nbr; ++k) {
            offs[(c * E + k) * 2] = nb[k][0];
            offs[(c * E + k) * 2 + 1] = nb[k][1];
            vals[(c * E + k) * 4] = t.coef[c][k];
          }
        }
        break;
      }
      case FSI_LAT_BT:
      case FSI_LAT_B: {
        fsi::DivTable<double> t;
        fsi::DivTable<float> tf;
        fsi::div_tables(n, t, tf);
        if (table == FSI_LAT_BT) {
          for (int c = 0; c < 4; ++c) {
            counts[c] = t.bt_count[c];
            for (int k = 0; k < t.bt_count[c]; ++k) {
              offs[(c * E + k) * 2] = t.bt_off[c][k][0];
              offs[(c * E + k) * 2 + 1] = t.bt_off[c][k][1];
              vals[(c * E + k) * 4] = t.bt_coef[c][k][0];
              vals[(c * E + k) * 4 + 1] = t.bt_coef[c][k][1];
            }
          }
        } else {
          counts[0] = t.b_count;
          for (int k = 0; k < t.b_count; ++k) {
            offs[k * 2] = t.b_off[k][0];
            offs[k * 2 + 1] = t.b_off[k][1];
            vals[k * 4] = t.b_coef[k][0];
            vals[k * 4 + 1] = t.b_coef[k][1];
          }
        }
        break;
      }
      case FSI_LAT_R: {
        fsi::P2RestrTable<double> t;
        fsi::P2RestrTable<float> tf;
        fsi::p2_restrict_tables(t, tf);
        for (int c = 0; c < 4; ++c) {
          counts[c] = t.count[c];
          for (int k = 0; k < t.count[c]; ++k) {
            offs[(c * E + k) * 2] = t.off[c][k][0];
            offs[(c * E + k) * 2 + 1] = t.off[c][k][1];
            vals[(c * E + k) * 4] = t.w[c][k];
          }
        }
        break;
      }
      case FSI_LAT_Q2AF: {
        fsi::Q2Table<double> t;
        fsi::Q2Table<float> tf;
        fsi::q2_tables(n, nu, rdt, t, tf);
        for (int c = 0; c < 4; ++c) {
          counts[c] = t.count[c];
          for (int k = 0; k < t.count[c]; ++k) {
            offs[(c * E + k) * 2] = t.off[c][k][0];
            offs[(c * E + k) * 2 + 1] = t.off[c][k][1];
            for (int q = 0; q < 4; ++q) vals[(c * E + k) * 4 + q] = t.coef[c][k][q];
          }
        }
        break;
      }
      default:
        throw Error(FSI_E_ARG, "unknown table id");
    }
  });
}

int fsi_export_csr(fsi_ctx *ctx, int block, int64_t *nrows, int64_t *nnz, int32_t *width,
                   int32_t *rowptr, int32_t *col, double *val) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    const fsi::Csr *A = nullptr;
    const double *v = nullptr;
    int w = 1;
    switch (block) {
      case FSI_BLK_AF: A = &c.Af; v = c.Af.val.p; w = 4; break;
      case FSI_BLK_MF: A = &c.Af; v = c.Mf.p; w = 1; break;
      case FSI_BLK_B: A = &c.B; v = c.B.val.p; w = 2; break;
      case FSI_BLK_BT: A = &c.BT; v = c.BT.val.p; w = 2; break;
      case FSI_BLK_AS: A = &c.S; v = c.S.val.p; w = 1; break;
      case FSI_BLK_CS: A = &c.S; v = c.Cs.p; w = 1; break;
      case FSI_BLK_CF: A = &c.Cf; v = c.Cf.val.p; w = 1; break;
      case FSI_BLK_CFT: A = &c.CfT; v = c.CfT.val.p; w = 1; break;
      case FSI_BLK_MP: A = &c.Mp; v = c.Mp.val.p; w = 1; break;
      case FSI_BLK_KT:
        FSI_REQUIRE(c.Kt.p, FSI_E_STATE, "no solid tangent: call fsi_solid_tangent");
        A = &c.S; v = c.Kt.p; w = 4; break;
      default: throw Error(FSI_E_ARG, "unknown block id");
    }
    if (block == FSI_BLK_CF || block == FSI_BLK_CFT)
      FSI_REQUIRE(c.have_cf, FSI_E_STATE, "call fsi_assemble_coupling first");
    if (nrows) *nrows = A->nrows;
    if (nnz) *nnz = A->nnz;
    if (width) *width = w;
    if (rowptr) FSI_HIP(hipMemcpyAsync(rowptr, A->rowptr.p, (A->nrows + 1) * 4, hipMemcpyDeviceToHost, c.stream));
    if (col && A->nnz) FSI_HIP(hipMemcpyAsync(col, A->col.p, A->nnz * 4, hipMemcpyDeviceToHost, c.stream));
    if (val && A->nnz) FSI_HIP(hipMemcpyAsync(val, v, A->nnz * w * 8, hipMemcpyDeviceToHost, c.stream));
    FSI_HIP(hipStreamSynchronize(c.stream));
  });
}

int fsi_profile(fsi_ctx *ctx, int enable) {
  if (!ctx) return FSI_E_ARG;
  Ctx &c = ctx->c;
  c.prof64.on = c.prof32.on = enable != 0;
  c.prof64.reset();
  c.prof32.reset();
  return FSI_OK;
}

int fsi_profile_read(fsi_ctx *ctx, int prec, int64_t *launches, double *total_ms,
                     double *bytes_per_launch) {
  if (!ctx) return FSI_E_ARG;
  return guarded(ctx, [&] {
    Ctx &c = ctx->c;
    FSI_REQUIRE(prec == FSI_FP64 || prec == FSI_FP32, FSI_E_ARG, "unknown precision");
    FSI_HIP(hipStreamSynchronize(c.stream));
    fsi::Prof &p = prec == FSI_FP64 ? c.prof64 : c.prof32;
    int64_t cnt = 0;
    double t = p.total_ms(cnt);
    const double w = prec == FSI_FP64 ? 8.0 : 4.0;
    const fsi::MgLevel &L = c.mgu.lv[0];
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = t;
    // FP32 form with three post-smoothing steps: the launch stores y into the FP64 output;
    // the direction is stored only for the single steps after the fused launch, which with
    // three or more steps also reads the coarse correction (two components, next level)
    const int degree = prec == FSI_FP64 ? c.mgu.degree : c.mgu.degree32;
    const double wy = (prec == FSI_FP32 && degree == 3) ? 8.0 : w;
    const double wd = degree > 3 ? w : 0.0;
    const double coarse = (degree >= 3 && c.mgu.lv.size() > 1) ? (double)c.mgu.lv[1].nodes * 2 * w : 0.0;
    // the class-stencil step of the Q2 pair: x, b and d read, d and y written (two components)
    if (bytes_per_launch)
      *bytes_per_launch = c.mgu.stencil ? (double)L.nodes * 2 * (2 * w + wd + wy) + coarse
                          : L.q2tab64.p ? (double)L.nodes * 2 * 5 * w
                                        : (double)L.A.nnz * (4 * w + 4) + (double)L.nodes * (4 + 14 * w) + 4.0;
  });
}

const char *fsi_strerror(int status) {
  switch (status) {
    case FSI_OK: return "ok";
    case FSI_E_ARG: return "invalid argument";
    case FSI_E_MESH: return "invalid mesh or solid position";
    case FSI_E_NOMEM: return "out of device memory or budget";
    case FSI_E_NOCONV: return "Krylov solve did not converge";
    case FSI_E_NONFINITE: return "non-finite value";
    case FSI_E_HIP: return "HIP runtime error";
    case FSI_E_CAPACITY: return "fixed capacity exceeded";
    case FSI_E_STATE: return "call order";
    default: return "unknown status";
  }
}

const char *fsi_last_error(const fsi_ctx *ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->c.last_error.c_str();
}

}  // extern "C"
