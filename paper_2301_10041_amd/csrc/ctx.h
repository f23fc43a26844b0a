// Internal state of a libfsi context and the host-side entry points of each module.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace fsi {

// CSR matrix with `width` values per entry (1: scalar, 2: (x, y) pair, 4: 2x2 block
// stored xx, xy, yx, yy).  FP64 master values and an FP32 shadow made on demand.
struct Csr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int width = 1;
  DevBuf<int> rowptr, col;
  DevBuf<double> val;
  DevBuf<float> val32;
  size_t bytes() const { return rowptr.bytes() + col.bytes() + val.bytes() + val32.bytes(); }
};

// Cells per side of the levels of the triangle pair's hierarchies on an n x n grid: halved
// while even and above 4 (the pressure levels, the last one solved densely).
inline std::vector<int> mg_level_cells(int n) {
  std::vector<int> ns;
  for (int m = n;; m /= 2) {
    ns.push_back(m);
    if (m <= 4 || (m & 1)) break;
  }
  return ns;
}
// Finest grid from which the velocity levels stop at the first coarse level of 16 x 16 cells
// or fewer, solved densely (a product with 2 (33)^2 = 2178 rows, 4.7 M words).  From 512^2 on
// that product reads at most a fifth of a cycle's words, and one wide launch beats the
// one-block coarse end (1024^2 FP64 step 130.9 -> 127.3 ms).  On smaller grids the levels go on
// to the last one: there the dense product would outweigh the rest of the cycle, and under
// concurrent systems its whole-chip launch costs more than the one-block coarse end (serving
// mix of 32^2 .. 256^2 grids: 166.6 -> 152.6 requests/s with the dense level everywhere).
constexpr int kDenseVelocityFromN = 512;
inline size_t mg_velocity_levels(const std::vector<int> &ns) {
  if (ns.size() < 2 || ns[0] < kDenseVelocityFromN) return ns.size();
  size_t nu = 1;
  while (nu + 1 < ns.size() && ns[nu] > 16) ++nu;
  return nu + 1;
}

// One level of a geometric multigrid hierarchy on the structured grid.
struct MgLevel {
  int n = 0;               // cells per side at this level
  int64_t nodes = 0;       // P2 nodes (velocity) or P1 nodes (pressure)
  Csr A;                   // operator (width 4 for velocity, 1 for pressure)
  DevBuf<double> dinv;     // inverse diagonal: 4 per node (2x2 blocks) or 1 per node
  DevBuf<float> dinv32;
  double lmax = 0.0;       // upper bound of the spectrum of D^{-1} A (power iteration x 1.1)
  Csr P, R;                // prolongation from the next coarser level into this one; R = P^T
  DevBuf<double> w64[5];   // x, b, r, d, x2 work vectors
  DevBuf<float> w32[5];
  DevBuf<unsigned char> stab64, stab32;   // StencilTable<double/float> (velocity levels)
  DevBuf<unsigned char> p1tab64, p1tab32; // P1Table<double/float> of L_p (pressure levels)
  DevBuf<unsigned char> q2tab64, q2tab32; // Q2Table<double/float> (velocity levels of the Q2 pair)
};

struct Mg {
  int comps = 1;           // unknowns per node: 2 (velocity, 2x2 blocks) or 1 (pressure)
  bool stencil = false;    // smoothing, residuals and transfers matrix-free (structured grid)
  bool tail = true;        // velocity levels of n <= 16 / pressure levels of n <= 64 in one launch
                           // (with the stencil form)
  int degree = 3;          // Chebyshev smoothing steps before and after the coarse correction
  int degree32 = 3;        // the same for the FP32 V-cycle of the mixed-precision form
  std::vector<MgLevel> lv; // lv[0] finest
  int64_t ncoarse = 0;     // unknowns of the coarsest level
  DevBuf<double> cinv;     // dense inverse of the coarsest operator (row major)
  DevBuf<float> cinv32;
  DevBuf<unsigned char> rtab64, rtab32;   // P2RestrTable<double/float> (velocity)
  size_t bytes() const;
};

// Event timing of one kernel class (pairs of events on the launching stream).
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  void begin(hipStream_t s);
  void end(hipStream_t s);
  double total_ms(int64_t &launches);
  void reset() { used = 0; }
  ~Prof();
};

struct Ctx {
  // problem
  int pair = FSI_PAIR_P2P1;   // element pair (fsi_create / fsi_create_q2)
  int n = 0;
  int device = 0;          // HIP device of the context (current at fsi_create)
  double nu = 1, rho = 1, dt = 0.01, kappa = 10;
  int64_t N2 = 0, Np = 0, Ns = 0, Nt = 0, N = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  std::string last_error;

  // fluid blocks on the finest grid
  Csr Af;                  // A_f with Dirichlet rows/columns, width 4
  DevBuf<double> Mf;       // M_f (no BC) on the A_f pattern, width 1
  Csr B;                   // B with BC and pin, width 2, rows P1
  Csr BT;                  // B^T, width 2, rows P2
  Csr Mp;                  // pressure mass, width 1
  DevBuf<double> Mp_dinv;  // 1 / diag(M_p)
  DevBuf<float> Mp_dinv32;
  DevBuf<unsigned char> mptab64, mptab32;  // P1Table<double/float> of M_p
  DevBuf<unsigned char> divtab64, divtab32;  // DivTable<double/float> (B and B^T)
  DevBuf<unsigned char> bnd;  // 1 on boundary P2 nodes

  // solid blocks
  std::vector<int> h_tri;  // host copy of the connectivity (3 per triangle; 4 per quadrilateral of the Q pair)
  std::vector<double> h_xy;
  DevBuf<int> tri;         // 3 per triangle
  DevBuf<double> ref_xy;   // [x | y]
  DevBuf<double> ref_area; // |E|
  DevBuf<int> n2e_ptr, n2e;// node -> 4*element + local vertex (sorted by element)
  int max_adj = 0;
  Csr S;                   // solid P1 pattern; val = A_s
  DevBuf<double> Cs;       // C_s on the same pattern
  DevBuf<float> Cs32;
  DevBuf<double> Cs_dinv;  // 1 / diag(C_s)
  // Chebyshev interval of D^{-1} C_s and the steps of the closed-form A22 solves: P1
  // triangles [1/2, 2], 36 steps; Q1 quadrilaterals [1/4, 9/4] (or the Gershgorin bound), 56
  double cs_lo = 0.5, cs_hi = 2.0;
  int cs_nsteps = 36;
  DevBuf<float> Cs_dinv32;
  // the S pattern transposed for coalesced row-per-lane reads: entry u of row r at u Ns + r,
  // rows padded to s_ew entries (column r, value 0); A_s and C_s values in the same order
  DevBuf<int> s_ecol;
  DevBuf<double> s_eas, s_ecs;
  int s_ew = 0;

  // coupling (rebuilt by every fsi_assemble_coupling)
  bool have_cf = false;
  bool pairs_kept = false; // the piece list (pair_E, pair_T) is in the context's buffers
  Csr Cf, CfT;
  int64_t n_pairs = 0, n_cand = 0;
  DevBuf<int> cand_off;    // Nt + 1
  DevBuf<int> piece_cnt;   // per candidate cell (then scanned in place, + 1)
  DevBuf<int> pair_E, pair_T;
  DevBuf<double> piece_L;  // 18 per piece: (|E|/|X(E)|) int lam_l phi_j
  DevBuf<int> e_piece;     // Nt + 1: first piece of each element
  DevBuf<int> cft_fill;     // C_f^T: per-row fill counters of the scatter
  DevBuf<int> cft_tcol;     // scattered (unordered) C_f^T rows before ranking
  DevBuf<double> cft_tval;
  DevBuf<int> cft_long;     // [count, rows...]: rows ranked by a workgroup each
  DevBuf<int> scan_tmp;     // scan partials (grow-only)
  DevBuf<int> cf_defer;     // [count, rows...]: C_f rows assembled with the wider windows
  DevBuf<int> cf_defer2;    // [count, rows...]: those above the middle window
  DevBuf<int> cf_huge;      // [count, largest window, rows...]: rows with a device-memory window
  DevBuf<int> cf_wflag;     // that window (grow-only)
  DevBuf<double> cf_wval;
  DevBuf<int> dflag;       // device error flags (mesh / capacity)
  int cf_hcnt[2] = {0, 0};  // rows with a device-memory window: count, largest window
  // the time-coherent form (FSI_COUPLING_INCREMENTAL): candidate boxes of (w + 1) x (h + 1)
  // cells, two piece slots per candidate (pair_T = -1 when empty), the positions of the last
  // call, and the permutation C_f^T entry -> C_f entry
  int cf_mode = FSI_COUPLING_FULL;
  bool inc_valid = false;   // the slots hold the pieces of the positions in inc_X
  DevBuf<int> inc_box;      // 2 Nt: box width and height in cells
  DevBuf<int> inc_moved;    // Nt
  DevBuf<int> inc_prevT;    // the slots' pieces before the last re-clip
  DevBuf<double> inc_X;     // 2 Ns
  DevBuf<int> inc_flag;     // [flags, moved elements, kept pieces, -]
  DevBuf<int> cft_tsrc;     // transpose staging: source entry of each scattered entry
  DevBuf<int> cft_perm;     // nnz: C_f entry of each C_f^T entry
  // calls, rebuilds, pattern rebuilds, value refills, unchanged (see fsi_coupling_counts)
  int64_t inc_counts[5] = {0, 0, 0, 0, 0};

  // multigrid hierarchies of the preconditioner
  Mg mgu, mgp;

  // Krylov work space (allocated on first use)
  struct Inner {
    DevBuf<double> v64[9];
    DevBuf<float> v32[9];
  } inner;
  struct Outer {
    int m = 0;
    int64_t ncap = 0;      // N the basis was allocated for
    DevBuf<double> V, Z, w, r, t, t2;
    DevBuf<float> x32, y32;
  } outer;
  DevBuf<double> red;      // reduction partials
  DevBuf<double> dscal;    // device scalars
  double *hpin = nullptr;  // pinned host staging (hipHostMalloc)
  // batched Arnoldi step (engine context): every system's dot products in one device buffer
  // and one pinned host copy of them
  DevBuf<double> bat_dh;
  double *bat_h = nullptr;
  size_t bat_h_n = 0;
  DevBuf<double> tmpN;     // N (operator/residual scratch)
  DevBuf<double> tmpS;     // 12 Ns (solid block scratch)

  // nonlinear solid (hyper.hip): the law, and its tangent K(X) on the solid pattern (2 x 2
  // blocks xx, xy, yx, yy) used in place of A_s by the operator and the preconditioners while
  // use_kt is set; Newton work vectors
  int law = FSI_LAW_LINEAR;
  double law_gamma = 0.0, law_eta = 0.0;
  bool use_kt = false;
  DevBuf<double> Kt;
  DevBuf<float> Kt32;
  DevBuf<double> nl_b, nl_r, nl_d, nl_R;

  Prof prof64, prof32;        // finest-level Chebyshev product on A_f

  // HIP graphs of the A11 preconditioner (one per precision), replayed on fixed staging
  // buffers; captured on first use, dropped when the smoother changes
  bool use_graphs = false;
  hipGraphExec_t pc_graph[2][FSI_MAX_LANES + 1] = {};   // per precision and lane count
  hipStream_t cap_stream = nullptr;   // capture only (default priority)
  // second stream of the A11 preconditioner: the pressure part (Schur approximation) runs
  // beside the velocity V-cycle, forked from and joined into the context stream by events
  // (default priority; created with the context)
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_ms[2] = {nullptr, nullptr};   // the inner MINRES state copies of two steps
  int ms_check = FSI_CHECK_AUTO;              // fsi_set_inner_check
  bool capturing = false;     // inside a graph capture: the preconditioner stays on one stream
  // inner MINRES: device-side scalar state, its own reduction buffer and solution vector
  // (allocated once: captured graphs hold these pointers), graphs per precision and phase
  DevBuf<double> ms_state, ms_red, ms_x, ms_part;
  DevBuf<double> ms_dot;   // per lane: velocity tile sums, then pressure block sums of r . z
  // the Lanczos vectors of the current block of iterations ([slot][lane][nf], ms_B slots),
  // the recorded direction scalars ([lane][slot][5]) and the combination coefficients
  DevBuf<double> ms_vh, ms_hist, ms_coef;
  int ms_B = 0;
  // inner GMRES (FSI_INNER_GMRES): basis, preconditioned vectors, reduction partials, device
  // results, scalars; pinned host staging
  DevBuf<double> gi_V, gi_Z, gi_part, gi_dh, gi_sc;
  double *gi_h = nullptr;
  double gi_wp = 0.0;   // weight of the pressure rows in its residual norm (set on first use)
  hipGraphExec_t ms_graph[2][FSI_MAX_LANES + 1][6] = {};   // per precision, lane count, rotation phase
  DevBuf<double> pc_in, pc_out;
  void drop_graphs();

  // systems the inner work space holds (lockstep solves of several contexts run their A11
  // solves on this context's lanes; lane stride = one system's vector length)
  int lanes = 1;
  double inner_rtol = -1.0;   // < 0: default per precision
  int inner_maxit = 1000;
  int inner_mode = FSI_INNER_MINRES;  // fsi_inner: how A11^{-1} is applied
  int inner_cycles = 1;               // FSI_INNER_FIXED_TRI: stationary cycles
  int64_t inner_its_total = 0;

  ~Ctx();
  size_t device_bytes() const;
};

// ---- module entry points (host side) ----
// assemble.hip
void build_fluid(Ctx &c);
void build_solid(Ctx &c);
void build_multigrid(Ctx &c);
void build_fluid_q2(Ctx &c);
void build_multigrid_q2(Ctx &c);
// coupling.hip
void assemble_coupling(Ctx &c, const double *Xn, bool sync_check);
void assemble_coupling_noalloc(Ctx &c, const double *Xn);
void assemble_coupling_q(Ctx &c, const double *Xn);
void reserve_coupling(Ctx &c);
void coupling_scratch_init(int dev);
// ops.hip (operator of eq. (matrix) and its pieces)
template <typename T, typename Tx>
void apply_operator(Ctx &c, const Tx *x, double *y, bool fluid_only);
void build_rhs(Ctx &c, const double *u_n, const double *X_n, double *b);
void make_shadow(Csr &A, hipStream_t s);
// solve.hip
void apply_precond(Ctx &c, int pc, int prec, const double *r, double *z);
void apply_precond_lanes(Ctx &engine, Ctx *const *cs, int K, int pc, int prec, const double *const *r,
                         double *const *z);
void gmres_solve(Ctx &c, const fsi_solve_opts &o, const double *b, double *x, fsi_solve_stats *st);
// hyper.hip
void solid_law(Ctx &c, const double *X, double *R, bool tangent);
void newton_step(Ctx &c, const fsi_solve_opts &o, const fsi_newton_opts &no, const double *u_n, const double *X_n,
                 const double *f_X, double *x, fsi_newton_stats *st);
void gmres_solve_lanes(Ctx *const *cs, int K, const fsi_solve_opts &o, const double *const *b,
                       double *const *x, fsi_solve_stats *st, int *rc);

}  // namespace fsi
