// Matrix-free pieces of the two multigrid hierarchies on the structured grid (see
// lattice.hip): P1 pressure operators (L_p with the pinned node, M_p), the first Chebyshev
// step with class-wise diagonal inverses, and the P2 / P1 grid transfers.
#pragma once

#include "common.h"
#include "stencil.h"

namespace fsi {

// P1 lattice (n + 1)^2 with the diagonal of each cell from (i, j) to (i + 1, j + 1): a node
// couples with itself and the six nodes at these offsets.
constexpr int kP1Nbr = 7;
// offsets: self, (-1,0), (+1,0), (0,-1), (0,+1), (-1,-1), (+1,+1)

// Node classes by position: ci = 0 (i = 0), 1 (interior), 2 (i = n); the same for j;
// class = 3 cj + ci.  coef[c][k] couples a node of class c with the node at offset k
// (zero where that node is outside the lattice).  pin = 1: the row of node 0 is the
// identity and its column is zero (the pressure level is fixed at node 0).
template <typename T>
struct P1Table {
  T coef[9][kP1Nbr];
  T dinv[9];
  int pin;
};

// P2 restriction R = P^T: for each class of coarse node (bit 0 = Ic odd, bit 1 = Jc odd),
// the fine nodes (offsets from the fine node 2 Ic, 2 Jc) whose interpolated value uses the
// coarse node, with the coarse basis function's value there as weight.
constexpr int kRestrMax = 81;
template <typename T>
struct P2RestrTable {
  int count[4];
  int off[4][kRestrMax][2];
  T w[4][kRestrMax];
};

// The fine-node offsets of the restriction classes in table order (dJ, then dI); they
// follow from the nested triangulation alone (the table builder checks them).  Kernels
// index them with compile-time class and entry.
constexpr int kRestrCount[4] = {25, 9, 9, 9};
struct RestrOffsets {
  int d[4][25][2];
};
__host__ __device__ constexpr RestrOffsets restrict_offsets() {
  return RestrOffsets{{
      {{-3, -3}, {-2, -3}, {-1, -3}, {0, -3}, {-3, -2}, {1, -2}, {-3, -1}, {-1, -1}, {0, -1},
       {2, -1}, {-3, 0}, {-1, 0}, {0, 0}, {1, 0}, {3, 0}, {-2, 1}, {0, 1}, {1, 1},
       {3, 1}, {-1, 2}, {3, 2}, {0, 3}, {1, 3}, {2, 3}, {3, 3}},
      {{-1, -2}, {-1, -1}, {0, -1}, {-1, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {1, 2}},
      {{-2, -1}, {-1, -1}, {0, -1}, {-1, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {2, 1}},
      {{-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {0, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1}},
  }};
}

// Lattice offsets (units h/2 from the cell's lower-left node) of the six P2 nodes of
// triangle t of a cell: T0 = (v00, v10, v11), T1 = (v00, v11, v01); vertices a, b, c
// then edge midpoints ab, bc, ca.
__host__ __device__ inline void p2_node_offset(int t, int b, int &dI, int &dJ) {
  const int vx[2][3] = {{0, 2, 2}, {0, 2, 0}};
  const int vy[2][3] = {{0, 0, 2}, {0, 2, 2}};
  if (b < 3) {
    dI = vx[t][b];
    dJ = vy[t][b];
  } else {
    const int p = b - 3, q = (p + 1) % 3;
    dI = (vx[t][p] + vx[t][q]) / 2;
    dJ = (vy[t][p] + vy[t][q]) / 2;
  }
}

// Coarse P2 interpolation at fine lattice node (I, J) of an nf grid (coarse grid nf / 2,
// nested): the coarse triangle holding the node, its barycentric coordinates (multiples of
// 1/4) and the non-zero values of the six coarse basis functions there.  Writes the coarse
// lattice coordinates and weights of up to 6 nodes; boundary nodes are not excluded.
__host__ __device__ inline int p2_prolong_weights(int I, int J, int nf, int *Ic, int *Jc, double *w) {
  const int nc = nf / 2;
  int ci = I / 4, cj = J / 4;
  if (ci > nc - 1) ci = nc - 1;
  if (cj > nc - 1) cj = nc - 1;
  const double xi = (I - 4 * ci) * 0.25, eta = (J - 4 * cj) * 0.25;
  int t;
  double l0, l1, l2;
  if (xi >= eta) {
    t = 0; l0 = 1.0 - xi; l1 = xi - eta; l2 = eta;
  } else {
    t = 1; l0 = 1.0 - eta; l1 = xi; l2 = eta - xi;
  }
  const double phi[6] = {l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                         4 * l0 * l1,       4 * l1 * l2,       4 * l2 * l0};
  int cnt = 0;
  for (int b = 0; b < 6; ++b) {
    if (phi[b] == 0.0) continue;
    int dI, dJ;
    p2_node_offset(t, b, dI, dJ);
    Ic[cnt] = 2 * ci + dI;
    Jc[cnt] = 2 * cj + dJ;
    w[cnt] = phi[b];
    ++cnt;
  }
  return cnt;
}

// Host table builders (which: kTableMp = pressure mass, kTableLp = pressure Laplacian)
constexpr int kTableMp = 216, kTableLp = 225;   // offsets of the P1 blocks in the element tables
void p1_tables(int n, int which, int pin, P1Table<double> &t64, P1Table<float> &t32);   // assemble.hip
void p2_restrict_tables(P2RestrTable<double> &t64, P2RestrTable<float> &t32);          // lattice.hip

// Launchers (stream-ordered, no synchronisation) over K independent systems (lane =
// blockIdx.y; each vector is a per-lane view, see LP; K = 1 for one system).  Vectors are
// component-major with the level's node count as stride.
template <typename T, int MODE>   // SP_APPLY, SP_RESID or SP_CHEB as for the A_f stencil
void p1_launch(int n, const P1Table<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c1, T c2,
               hipStream_t s, int K = 1);
// d = x = scale D^{-1} b (first Chebyshev step from zero), class-wise diagonal
template <typename T>
void p1_first(int n, const P1Table<T> *tab, LP<const T> b, T scale, LP<T> d, LP<T> x, hipStream_t s, int K = 1);
template <typename T>
void p2_first(int n, const StencilTable<T> *tab, LP<const T> b, T scale, LP<T> d, LP<T> x, hipStream_t s,
              int K = 1);
// y += P xc (fine grid nf; coarse vector on the nf / 2 grid); P2 has two components
template <typename T>
void p2_prolong_add(int nf, LP<const T> xc, LP<T> y, hipStream_t s, int K = 1);
template <typename T>
void p1_prolong_add(int nf, LP<const T> xc, LP<T> y, hipStream_t s, int K = 1);
// bc = R r (pressure levels; the velocity levels restrict in resid_restrict)
template <typename T>
void p1_restrict(int nf, LP<const T> r, LP<T> bc, hipStream_t s, int K = 1);
// S Chebyshev steps on a P1 operator in one launch (lattice.hip, k_p1_multi): from zero or
// from x, the result to y or combined into the Schur output z = a x + b2 w (pinned entry
// r[0], per-tile parts of sum r z).  Lane strides: lb for b, x, y, w; lz for z, r, r64; lp
// for part (p1_multi_tiles(n) parts per lane).
constexpr int kP1T = 16, kP1C = 64;   // tile rows and columns (256 threads)
enum { P1_OUT_X = 0, P1_OUT_SCHUR = 1 };
template <typename T, typename TZ>
struct P1MultiArgs {
  int n;
  const P1Table<T> *tab;
  const T *b, *x;
  T *y;
  T c1[3], c2[3];   // step k: d = c1[k] d + c2[k] D^{-1} (b - A x); from zero c2[0] scales D^{-1} b
  TZ *z;
  const TZ *r;
  const double *r64;
  const T *w;
  T a, b2;
  double *part;
  int64_t lb, lz, lp;
};
int p1_multi_tiles(int n);
template <typename T, typename TZ, int S, bool ZERO, int OUT>
void p1_multi(const P1MultiArgs<T, TZ> &a, hipStream_t s, int K = 1);
// The coarse end of a velocity V-cycle in one launch per system (mgtail.hip): levels
// lv[0..nlev) (n <= kTailMaxN cells, each the next one's fine level) and the coarsest
// level's dense inverse.  Vectors in LDS (offsets in T): level l's b at lv[l].off and x
// right after it (2 N each, N = tail_plane_entries(n)), one shared direction at offd (2 N of
// lv[0]),
// the coarsest b at offc and x after it (m each), then the stencil coefficients and
// inverse diagonal blocks of every level (kTailTab each) and the restriction weights
// (kTailRw) at offt; the dense inverse of the coarsest level (m x m, row-major) at offm when
// it fits the block's LDS, else offm = -1 and it is read from device memory; lds = the
// total.  b and x in device memory: the first level's right-hand side and result (lane
// stride lb).
constexpr int kTailMax = 4, kTailDeg = 8, kTailMaxN = 16, kTailDenseMax = 6 * 64;
constexpr int kTailCoef[4] = {0, 76, 112, 148};   // class offsets of 4 coefficients per entry
constexpr int kTailTab = 184 + 16, kTailRw = 25 + 9 + 9 + 9;
constexpr int kTailRs[4] = {0, 25, 34, 43};       // class offsets of the restriction weights
// Largest LDS block of the tail launch on the current device (queried once, at most 160 KiB).
int tail_lds_limit();
// Entries per component of a smoothing level of n cells in the tail's LDS: even and odd
// column planes of n + 1 columns and 2n + 1 rows.
inline int tail_plane_entries(int n) { return 2 * (2 * n + 1) * (n + 1); }
template <typename T>
struct TailLevel {
  int n, off;
  const StencilTable<T> *tab;
  T s;                                     // 1 / theta: the first step of both smoothings
  T c1[kTailDeg - 1], c2[kTailDeg - 1];    // the later Chebyshev steps
};
template <typename T>
struct TailArgs {
  int nlev, degree;
  TailLevel<T> lv[kTailMax];
  int offd, offc, offt, offm, m, lds;
  const P2RestrTable<T> *rt;
  const T *cinv;
  const T *b;
  T *x;
  int64_t lb;
};
template <typename T>
void mg_tail(const TailArgs<T> &a, hipStream_t s, int K = 1);
// The coarse end of a pressure (P1) V-cycle in one launch per system (mgtail.hip): levels
// lv[0..nlev) of at most kPTailMaxN cells (each the next one's fine level) and the dense
// inverse of the coarsest.  LDS (offsets in T): level l's b at lv[l].off and x right after it
// ((n + 1)^2 each, row-major), a shared second iterate at offx2 ((n + 1)^2 of lv[0]: the
// ping-pong buffer of the smoothing steps, then the residual), the coarsest b at offc and x
// after it (m each), the P1 tables of the levels (kPTailTab each) at offt, and the dense
// inverse at offm when it fits (else offm = -1: read from device memory); lds = the total.
// b and x in device memory: the first level's right-hand side and result (lane stride lb).
// Each node's search direction stays in a register of the thread that owns it
// (kPTailPer nodes per thread).
constexpr int kPTailMax = 6, kPTailDeg = 4, kPTailMaxN = 64, kPTailPer = 5, kPTailDenseMax = 6 * 64;
constexpr int kPTailTab = 9 * kP1Nbr + 9;   // coef[9][7], dinv[9]
template <typename T>
struct PTailLevel {
  int n, off;
  const P1Table<T> *tab;
  T c1[kPTailDeg], c2[kPTailDeg];   // p1_cheb_coefs of the level
};
template <typename T>
struct PTailArgs {
  int nlev, degree;
  PTailLevel<T> lv[kPTailMax];
  int offx2, offc, offt, offm, m, lds;
  const T *cinv;
  const T *b;
  T *x;
  int64_t lb;
};
template <typename T>
void p1_tail(const PTailArgs<T> &a, hipStream_t s, int K = 1);
// bc = R (b - A_f x) in one launch (stencil.hip): the residual lives only in LDS
template <typename T>
void resid_restrict(int nf, const StencilTable<T> *tab, const P2RestrTable<T> *rtab, LP<const T> x,
                    LP<const T> b, LP<T> bc, hipStream_t s, int K = 1);

}  // namespace fsi
