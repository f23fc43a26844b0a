// The velocity operator of the paper's element pair (Q2 on the n x n squares) in class form:
// an interior Q2 node of class c = (I & 1) + 2 (J & 1) (vertex, x-edge midpoint, y-edge midpoint,
// centre) couples with the nodes of the 4, 2, 2 or 1 cells around it (25, 15, 15 or 9 offsets in
// [-2, 2]^2); every interior row of A_f = (rho/dt) M_f + K_f is the class's stencil with the
// Dirichlet neighbours left out, and a boundary row is the identity.
#pragma once

#include <vector>

#include "common.h"

namespace fsi {

constexpr int kQ2Max = 25;

// Element table of the pair on a cell of side 1/n (assemble.hip): M (9 x 9) at QE_M,
// K[alpha][beta] (nu eps(phi_j e_beta) : eps(phi_i e_alpha), 4 x 9 x 9) at QE_K, B[alpha][k]
// (2 x 3 x 9) at QE_B, the diagonal of M_p (3) at QE_MP
constexpr int QE_M = 0, QE_K = 81, QE_B = QE_K + 324, QE_MP = QE_B + 54, QE_SIZE = QE_MP + 3;
void q2_element_table(int n, double nu, std::vector<double> &out);

template <typename T>
struct Q2Table {
  int count[4];
  int off[4][kQ2Max][2];   // (dI, dJ), dJ major
  T coef[4][kQ2Max][4];    // 2 x 2 blocks: xx, xy, yx, yy
  T dinv[4][4];            // inverse of the diagonal block
  T dense[4][25][4];       // the same blocks on the full 5 x 5 window, entry (dI + 2) + 5 (dJ + 2) (zero
                           // where the class has no neighbour)
};

// One pass over the velocity lattice of an n x n grid (components at x and x + (2n+1)^2):
//   resid: y = b - A x
//   else:  d = c1 d + c2 D^{-1} (b - A x), y = x + d   (a Chebyshev step)
template <typename T>
void q2_stencil(int n, const Q2Table<T> *tab, const T *x, const T *b, T *d, T *y, T c1, T c2, bool resid,
                hipStream_t s);

// Host: the class stencils of A_f on an n x n grid (n >= 2) from the Q2 element matrices.
void q2_tables(int n, double nu, double rdt, Q2Table<double> &t64, Q2Table<float> &t32);

}  // namespace fsi
