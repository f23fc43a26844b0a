// Coefficient tables of the matrix-free A_f products (see stencil.hip).
#pragma once

#include "common.h"

namespace fsi {

constexpr int kStencilMax = 25;   // a P2 node couples with at most 19 nodes (5 x 5 window)
constexpr int kTileC = 128;       // tile of the tiled kernel: kTileR lattice rows x kTileC nodes
constexpr int kTileR = 4;

// Node classes: bit 0 = I odd, bit 1 = J odd (0 vertex, 1 horizontal edge, 2 vertical
// edge, 3 diagonal edge).  coef[c][k] is the 2x2 block (xx, xy, yx, yy) of A_f coupling a
// node of class c with the node at lattice offset off[c][k]; dinv[c] is the inverse of the
// diagonal block.
template <typename T>
struct StencilTable {
  int count[4];
  int off[4][kStencilMax][2];
  int lin[4][kStencilMax];       // dJ (2n+1) + dI: offset of the neighbour's index
  int lds[4][kStencilMax];       // dJ (kTileC + 4) + dI: offset inside the LDS tile
  T coef[4][kStencilMax][4];
  T dinv[4][4];
};

// Neighbour counts of the classes on the triangulated grid (vertex, h-edge, v-edge, diagonal).
constexpr int kStencilCount[4] = {19, 9, 9, 9};

// The neighbour offsets (dI, dJ) of each class, in the order of the tables (dJ, then dI,
// ascending).  They follow from the triangulation alone; the table builder checks them.
// Kernels index them with compile-time class and neighbour, so LDS addresses become
// instruction immediates.
struct StencilOffsets {
  int d[4][kStencilMax][2];
};
__host__ __device__ constexpr StencilOffsets stencil_offsets() {
  return StencilOffsets{{
      {{-2, -2}, {-1, -2}, {0, -2}, {-2, -1}, {-1, -1}, {0, -1}, {1, -1}, {-2, 0}, {-1, 0}, {0, 0},
       {1, 0}, {2, 0}, {-1, 1}, {0, 1}, {1, 1}, {2, 1}, {0, 2}, {1, 2}, {2, 2}},
      {{-1, -2}, {-1, -1}, {0, -1}, {-1, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {1, 2}},
      {{-2, -1}, {-1, -1}, {0, -1}, {-1, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {2, 1}},
      {{-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {0, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1}},
  }};
}

// Entries whose cross-component couplings (xy, yx) vanish for every viscosity and time step:
// the symmetric-gradient form couples the components only through mixed derivatives, which
// integrate to zero for these neighbour pairs on the triangulated grid (the table builder
// checks that both values are exactly 0).  Kernels skip their two cross products.
struct CrossZero {
  bool z[4][kStencilMax];
};
__host__ __device__ constexpr CrossZero cross_zero() {
  CrossZero c{};
  c.z[0][1] = c.z[0][3] = c.z[0][15] = c.z[0][17] = true;   // vertex: (-1,-2), (-2,-1), (2,1), (1,2)
  c.z[1][0] = c.z[1][8] = true;                              // horizontal edge: (-1,-2), (1,2)
  c.z[2][0] = c.z[2][8] = true;                              // vertical edge: (-2,-1), (2,1)
  return c;
}

// Divergence blocks on the structured grid.  B^T row of an interior P2 node of class c:
// the P1 vertices of the triangles around it (offsets from P1 node (I >> 1, J >> 1)) with
// the pair (B_x, B_y)(k, node).  B row of a P1 node (i, j): the P2 nodes of the triangles
// around it (lattice offsets from (2i, 2j)).  Rows of Dirichlet P2 nodes of B^T and the
// matching columns of B are zero; so are row 0 of B and column 0 of B^T (pinned pressure).
// Every triangle holding an interior P2 node lies in the domain, so one B row serves every
// P1 node, boundary ones included, once the Dirichlet values of x_u are read as zero.
constexpr int kBtMax = 7;
constexpr int kBMax = 19;
constexpr int kBtCount[4] = {7, 4, 4, 4};
// Entry order of both tables: by dJ, then dI (the builder sorts and checks).  B^T offsets
// are P1 lattice offsets from (I >> 1, J >> 1); B offsets are P2 lattice offsets from
// (2i, 2j), the pattern of the vertex class of A_f.
struct DivOffsets {
  int bt[4][kBtMax][2];
};
__host__ __device__ constexpr DivOffsets div_offsets() {
  return DivOffsets{{
      {{-1, -1}, {0, -1}, {-1, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}},
      {{0, -1}, {0, 0}, {1, 0}, {1, 1}},
      {{-1, 0}, {0, 0}, {0, 1}, {1, 1}},
      {{0, 0}, {1, 0}, {0, 1}, {1, 1}},
  }};
}
template <typename T>
struct DivTable {
  int bt_count[4];
  int bt_off[4][kBtMax][2];
  T bt_coef[4][kBtMax][2];
  int b_count;
  int b_off[kBMax][2];
  int b_lds[kBMax];              // dJ (kTileC + 4) + dI
  T b_coef[kBMax][2];
};

// Launchers run K independent systems (lane = blockIdx.y) over per-lane views (LP); the
// vector views of one launch share one lane stride.  K = 1: one system.
template <typename T, int MODE>
void stencil_launch(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c1,
                    T c2, hipStream_t s, int K = 1);

// Fluid rows of the operator on [u_x | u_y | p] in one tiled launch:
//   y_u = A_f x_u - B^T x_p (+ C_f^T x_lam when cft_rp is given; lam_x at xl, lam_y at xl + Ns)
//   y_p = -B x_u, and y_p[0] = x_p[0] (pinned node)
template <typename T>
void stencil_fluid_rows(int n, const StencilTable<T> *tab, const DivTable<T> *dv, const T *x, T *y,
                        const int *cft_rp, const int *cft_col, const T *cft_val, const T *xl, int64_t Ns,
                        hipStream_t s);

// Two Chebyshev steps per launch on the A_f stencil (temporal blocking):
// cheb2_pre : x = d = s D^{-1} b, then two steps (c1a, c2a), (c1b, c2b); writes x, d
// cheb2_post: from x, a step with c1 = 0 (c2a) and a step (c1b, c2b); writes y, d
// (all three: a null d skips the store of the last direction when no later step reads it)
template <typename T>
void cheb2_pre(int n, const StencilTable<T> *tab, LP<const T> b, LP<T> d, LP<T> x, T s, T c1a, T c2a, T c1b,
               T c2b, hipStream_t st, int K = 1);
template <typename T>
void cheb2_post(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c2a, T c1b,
                T c2b, hipStream_t st, int K = 1);
// cheb3_post: from x, a step with c1 = 0 (c2a) and steps (c1b, c2b), (c1c, c2c); writes y
// (stored as TY: double or T) and d.  With xc (coarse lattice n / 2, same lane count) the
// steps start from x + P xc (the V-cycle's coarse correction; x itself is not written).
// With dot, tile t of lane k stores the sum over its nodes of b . y (FP64, y as stored) at
// dot.at(k)[t] (cheb3_dot_count(n) tiles); with b64 the sums take that FP64 right-hand side
// in place of b (the FP32 cycle of the mixed form).
template <typename T, typename TY = T>
void cheb3_post(int n, const StencilTable<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<TY> y, T c2a, T c1b,
                T c2b, T c1c, T c2c, hipStream_t st, int K = 1, LP<const T> xc = LP<const T>(),
                LP<double> dot = LP<double>(), LP<const double> b64 = LP<const double>());
int cheb3_dot_count(int n);

// The same launch inside the inner MINRES (FP64): v = s x, y = s (A11 x) + c r1 written over
// r1, and one partial sum of v . y per tile in part[] (s, c read from device memory;
// r1 read only when c != 0).  v goes to slot *slot_dev (a device scalar, clamped to
// [0, nslot - 1]) of the Lanczos block: v.p + slot vs + lane v.s.  Returns the number of
// tiles (entries of part per lane).
int stencil_a11_minres(int n, const StencilTable<double> *tab, const DivTable<double> *dv, LP<const double> x,
                       LP<double> v, LP<double> r1y, LP<const double> s_dev, LP<const double> c_dev,
                       LP<const double> slot_dev, int64_t vs, int nslot, LP<double> part, hipStream_t s,
                       int K = 1);
int stencil_tile_count(int n);

// Host: the tables of A_f on an n x n grid from the element matrices (assemble.hip).
void stencil_tables(int n, double nu, double rdt, StencilTable<double> &t64, StencilTable<float> &t32);
void div_tables(int n, DivTable<double> &t64, DivTable<float> &t32);

}  // namespace fsi
