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

template <typename T, int MODE>
void stencil_launch(int n, const StencilTable<T> *tab, const T *x, const T *b, T *d, T *y, T c1, T c2,
                    hipStream_t s);

template <typename T>
void stencil_a11_velocity(int n, const StencilTable<T> *tab, const int *bt_rp, const int *bt_col,
                          const T *bt_val, const T *x, T *y, hipStream_t s);

// Host: the tables of A_f on an n x n grid from the element matrices (assemble.hip).
void stencil_tables(int n, double nu, double rdt, StencilTable<double> &t64, StencilTable<float> &t32);

}  // namespace fsi
