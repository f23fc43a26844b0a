// Assembly of the time-independent blocks of eq. (matrix) (Sec. 4) on the device:
//   A_f = (rho/dt) M_f + K_f (2x2 blocks, K_f from nu (eps(u), eps(v))), M_f, B (div),
//   B^T, the pressure mass M_p and the P1 pressure Laplacian L_p (preconditioner);
//   A_s = kappa K_s and C_s = M_s on the solid mesh;
// and the geometric multigrid hierarchies (P2 velocity, P1 pressure) with nested
// prolongations.  Every matrix row is gathered by one thread from the triangles around
// its node, so there are no atomics and the result is deterministic.  Columns of a row
// are visited in a fixed window order that coincides with ascending node index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ctx.h"
#include "kernels.h"
#include "lattice.h"
#include "q2.h"
#include "stencil.h"

namespace fsi {

// Copy of a host table into a device buffer (synchronous: the host object is a local).
static void upload_bytes(DevBuf<unsigned char> &dst, const void *src, size_t bytes, hipStream_t s) {
  dst.alloc(bytes);
  FSI_HIP(hipMemcpyAsync(dst.p, src, bytes, hipMemcpyHostToDevice, s));
  FSI_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- element matrices
// Degree-4 six-point rule on a triangle (Dunavant, 1985): positive weights, exact for
// polynomials of degree <= 4, which covers every integrand below (P2 x P2 mass).
static const double kDunA[2] = {0.445948490915965, 0.091576213509771};
static const double kDunW[2] = {0.223381589678011, 0.109951743655322};

// Layout of one element type in the device table.
constexpr int EM_M = 0, EM_K = 36, EM_B = 180, EM_MP = 216, EM_LP = 225, EM_SIZE = 234;
static_assert(EM_MP == kTableMp && EM_LP == kTableLp, "P1 table ids are the element-table offsets");

// Lattice offsets of the six P2 nodes (a, b, c, ab, bc, ca) of the two triangles of a
// cell, in units of h/2 from the cell's lower-left node (2i, 2j).
__constant__ int kOff[2][6][2] = {{{0, 0}, {2, 0}, {2, 2}, {1, 0}, {2, 1}, {1, 1}},
                                  {{0, 0}, {2, 2}, {0, 2}, {1, 1}, {1, 2}, {0, 1}}};
static const int hOff[2][6][2] = {{{0, 0}, {2, 0}, {2, 2}, {1, 0}, {2, 1}, {1, 1}},
                                  {{0, 0}, {2, 2}, {0, 2}, {1, 1}, {1, 2}, {0, 1}}};

// Element matrices of T0 = (v00, v10, v11) and T1 = (v00, v11, v01) of a cell of side h.
static void element_tables(int n, double nu, std::vector<double> &out) {
  const double h = 1.0 / n;
  const double area = 0.5 * h * h;
  out.assign(2 * EM_SIZE, 0.0);
  for (int t = 0; t < 2; ++t) {
    // barycentric gradients (constant on the triangle)
    double g[3][2];
    if (t == 0) {   // l0 = 1 - xi, l1 = xi - eta, l2 = eta
      g[0][0] = -1 / h; g[0][1] = 0;
      g[1][0] = 1 / h;  g[1][1] = -1 / h;
      g[2][0] = 0;      g[2][1] = 1 / h;
    } else {        // l0 = 1 - eta, l1 = xi, l2 = eta - xi
      g[0][0] = 0;      g[0][1] = -1 / h;
      g[1][0] = 1 / h;  g[1][1] = 0;
      g[2][0] = -1 / h; g[2][1] = 1 / h;
    }
    double *E = out.data() + t * EM_SIZE;
    for (int q = 0; q < 6; ++q) {
      int grp = q / 3, rot = q % 3;
      double a = kDunA[grp], b = 1.0 - 2.0 * a;
      double l[3];
      l[rot] = b; l[(rot + 1) % 3] = a; l[(rot + 2) % 3] = a;
      double w = kDunW[grp] * area;
      static const int ea[3] = {0, 1, 2}, eb[3] = {1, 2, 0};
      double phi[6], dphi[6][2];
      for (int k = 0; k < 3; ++k) {
        phi[k] = l[k] * (2 * l[k] - 1);
        for (int c = 0; c < 2; ++c) dphi[k][c] = (4 * l[k] - 1) * g[k][c];
      }
      for (int k = 0; k < 3; ++k) {
        int p = ea[k], r = eb[k];
        phi[3 + k] = 4 * l[p] * l[r];
        for (int c = 0; c < 2; ++c) dphi[3 + k][c] = 4 * (l[r] * g[p][c] + l[p] * g[r][c]);
      }
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
          E[EM_M + i * 6 + j] += w * phi[i] * phi[j];
          double gg = dphi[i][0] * dphi[j][0] + dphi[i][1] * dphi[j][1];
          // eps(phi_j e_beta) : eps(phi_i e_alpha) = (delta_ab grad phi_i . grad phi_j
          //                                           + d_beta phi_i d_alpha phi_j) / 2
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be)
              E[EM_K + ((al * 2 + be) * 6 + i) * 6 + j] +=
                  w * nu * 0.5 * ((al == be ? gg : 0.0) + dphi[i][be] * dphi[j][al]);
        }
      for (int al = 0; al < 2; ++al)
        for (int k = 0; k < 3; ++k)
          for (int i = 0; i < 6; ++i) E[EM_B + (al * 3 + k) * 6 + i] += w * dphi[i][al] * l[k];
      for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) {
          E[EM_MP + k * 3 + m] += w * l[k] * l[m];
          E[EM_LP + k * 3 + m] += w * (g[k][0] * g[m][0] + g[k][1] * g[m][1]);
        }
    }
  }
}

__global__ void k_diag_inv(int64_t nrows, const int *rowptr, const int *col, const double *v,
                           double *dinv);

// Host: rows of A_f at one interior node of each class, gathered like k_asm_p2p2 (the same
// window order and the same order of triangles), with offsets relative to the node.
void stencil_tables(int n, double nu, double rdt, StencilTable<double> &t64, StencilTable<float> &t32) {
  FSI_REQUIRE(n >= 2, FSI_E_ARG, "stencil tables need n >= 2");
  std::vector<double> E;
  element_tables(n, nu, E);
  std::memset(&t64, 0, sizeof(t64));
  std::memset(&t32, 0, sizeof(t32));
  for (int cls = 0; cls < 4; ++cls) {
    const int I = 2 + (cls & 1), J = 2 + ((cls >> 1) & 1);   // interior for n >= 2
    struct A { int ci, cj, t, a; } adj[8];
    int na = 0;
    for (int cj = std::max(0, (J - 1) >> 1); cj <= std::min(n - 1, J >> 1); ++cj)
      for (int ci = std::max(0, (I - 1) >> 1); ci <= std::min(n - 1, I >> 1); ++ci)
        for (int t = 0; t < 2; ++t)
          for (int a = 0; a < 6; ++a)
            if (2 * ci + hOff[t][a][0] == I && 2 * cj + hOff[t][a][1] == J) {
              adj[na++] = A{ci, cj, t, a};
              break;
            }
    int cnt = 0;
    for (int dJ = -2; dJ <= 2; ++dJ)
      for (int dI = -2; dI <= 2; ++dI) {
        bool touched = false;
        double m = 0, kxx = 0, kxy = 0, kyx = 0, kyy = 0;
        for (int q = 0; q < na; ++q) {
          int b = -1;
          for (int bb = 0; bb < 6; ++bb)
            if (2 * adj[q].ci + hOff[adj[q].t][bb][0] == I + dI && 2 * adj[q].cj + hOff[adj[q].t][bb][1] == J + dJ) b = bb;
          if (b < 0) continue;
          touched = true;
          const double *e = E.data() + adj[q].t * EM_SIZE;
          const int a = adj[q].a;
          m += e[EM_M + a * 6 + b];
          kxx += e[EM_K + ((0 * 2 + 0) * 6 + a) * 6 + b];
          kxy += e[EM_K + ((0 * 2 + 1) * 6 + a) * 6 + b];
          kyx += e[EM_K + ((1 * 2 + 0) * 6 + a) * 6 + b];
          kyy += e[EM_K + ((1 * 2 + 1) * 6 + a) * 6 + b];
        }
        if (!touched) continue;
        FSI_REQUIRE(cnt < kStencilMax, FSI_E_ARG, "stencil too wide");
        double v[4] = {rdt * m + kxx, kxy, kyx, rdt * m + kyy};
        t64.off[cls][cnt][0] = t32.off[cls][cnt][0] = dI;
        t64.off[cls][cnt][1] = t32.off[cls][cnt][1] = dJ;
        t64.lin[cls][cnt] = t32.lin[cls][cnt] = dJ * (2 * n + 1) + dI;
        t64.lds[cls][cnt] = t32.lds[cls][cnt] = dJ * (kTileC + 4) + dI;
        for (int q = 0; q < 4; ++q) {
          t64.coef[cls][cnt][q] = v[q];
          t32.coef[cls][cnt][q] = (float)v[q];
        }
        if (dI == 0 && dJ == 0) {
          double det = v[0] * v[3] - v[1] * v[2];
          double di[4] = {v[3] / det, -v[1] / det, -v[2] / det, v[0] / det};
          for (int q = 0; q < 4; ++q) {
            t64.dinv[cls][q] = di[q];
            t32.dinv[cls][q] = (float)di[q];
          }
        }
        ++cnt;
      }
    t64.count[cls] = t32.count[cls] = cnt;
    FSI_REQUIRE(cnt == kStencilCount[cls], FSI_E_ARG, "unexpected stencil width");
    constexpr StencilOffsets so = stencil_offsets();
    for (int k = 0; k < cnt; ++k)
      FSI_REQUIRE(t64.off[cls][k][0] == so.d[cls][k][0] && t64.off[cls][k][1] == so.d[cls][k][1], FSI_E_ARG,
                  "stencil offsets differ from the compiled pattern");
    constexpr CrossZero cz = cross_zero();
    for (int k = 0; k < cnt; ++k)
      FSI_REQUIRE(!cz.z[cls][k] || (t64.coef[cls][k][1] == 0.0 && t64.coef[cls][k][2] == 0.0), FSI_E_ARG,
                  "a cross coupling compiled as zero is not");
  }
}

// Host: B^T rows of the four interior P2 node classes and the B row of an interior P1
// node, summed over the triangles around the node from the element blocks
// B_alpha(k, i) = int d_alpha phi_i lam_k.
void div_tables(int n, DivTable<double> &t64, DivTable<float> &t32) {
  FSI_REQUIRE(n >= 2, FSI_E_ARG, "divergence tables need n >= 2");
  std::vector<double> E;
  element_tables(n, 1.0, E);
  std::memset(&t64, 0, sizeof(t64));
  std::memset(&t32, 0, sizeof(t32));
  struct A { int ci, cj, t, a; };
  auto around = [&](int I, int J, A *adj) {
    int na = 0;
    for (int cj = std::max(0, (J - 1) >> 1); cj <= std::min(n - 1, J >> 1); ++cj)
      for (int ci = std::max(0, (I - 1) >> 1); ci <= std::min(n - 1, I >> 1); ++ci)
        for (int t = 0; t < 2; ++t)
          for (int a = 0; a < 6; ++a)
            if (2 * ci + hOff[t][a][0] == I && 2 * cj + hOff[t][a][1] == J) {
              adj[na++] = A{ci, cj, t, a};
              break;
            }
    return na;
  };
  A adj[8];
  for (int cls = 0; cls < 4; ++cls) {
    const int I = 2 + (cls & 1), J = 2 + (cls >> 1);
    const int na = around(I, J, adj);
    int cnt = 0;
    for (int q = 0; q < na; ++q)
      for (int v = 0; v < 3; ++v) {   // P1 vertex v of the triangle
        const int di = (2 * adj[q].ci + hOff[adj[q].t][v][0]) / 2 - (I >> 1);
        const int dj = (2 * adj[q].cj + hOff[adj[q].t][v][1]) / 2 - (J >> 1);
        int k = 0;
        while (k < cnt && !(t64.bt_off[cls][k][0] == di && t64.bt_off[cls][k][1] == dj)) ++k;
        if (k == cnt) {
          FSI_REQUIRE(cnt < kBtMax, FSI_E_ARG, "B^T stencil too wide");
          t64.bt_off[cls][k][0] = t32.bt_off[cls][k][0] = di;
          t64.bt_off[cls][k][1] = t32.bt_off[cls][k][1] = dj;
          ++cnt;
        }
        const double *e = E.data() + adj[q].t * EM_SIZE + EM_B;
        for (int al = 0; al < 2; ++al) t64.bt_coef[cls][k][al] += e[(al * 3 + v) * 6 + adj[q].a];
      }
    t64.bt_count[cls] = t32.bt_count[cls] = cnt;
  }
  {
    const int na = around(2, 2, adj);   // P1 node (1, 1)
    int cnt = 0;
    for (int q = 0; q < na; ++q) {
      FSI_REQUIRE(adj[q].a < 3, FSI_E_ARG, "P1 node is not a vertex");
      for (int b = 0; b < 6; ++b) {
        const int dI = 2 * adj[q].ci + hOff[adj[q].t][b][0] - 2, dJ = 2 * adj[q].cj + hOff[adj[q].t][b][1] - 2;
        int k = 0;
        while (k < cnt && !(t64.b_off[k][0] == dI && t64.b_off[k][1] == dJ)) ++k;
        if (k == cnt) {
          FSI_REQUIRE(cnt < kBMax, FSI_E_ARG, "B stencil too wide");
          t64.b_off[k][0] = t32.b_off[k][0] = dI;
          t64.b_off[k][1] = t32.b_off[k][1] = dJ;
          t64.b_lds[k] = t32.b_lds[k] = dJ * (kTileC + 4) + dI;
          ++cnt;
        }
        const double *e = E.data() + adj[q].t * EM_SIZE + EM_B;
        for (int al = 0; al < 2; ++al) t64.b_coef[k][al] += e[(al * 3 + adj[q].a) * 6 + b];
      }
    }
    t64.b_count = t32.b_count = cnt;
  }
  // canonical order (dJ, then dI), checked against the offsets the kernels are compiled with
  auto sort_entries = [](int cnt, int (*off)[2], double (*coef)[2], int *lds) {
    for (int a = 1; a < cnt; ++a)
      for (int b = a; b > 0; --b) {
        const bool less = off[b][1] < off[b - 1][1] || (off[b][1] == off[b - 1][1] && off[b][0] < off[b - 1][0]);
        if (!less) break;
        std::swap(off[b][0], off[b - 1][0]);
        std::swap(off[b][1], off[b - 1][1]);
        std::swap(coef[b][0], coef[b - 1][0]);
        std::swap(coef[b][1], coef[b - 1][1]);
        if (lds) std::swap(lds[b], lds[b - 1]);
      }
  };
  constexpr DivOffsets dofs = div_offsets();
  constexpr StencilOffsets sofs = stencil_offsets();
  for (int c = 0; c < 4; ++c) {
    sort_entries(t64.bt_count[c], t64.bt_off[c], t64.bt_coef[c], nullptr);
    FSI_REQUIRE(t64.bt_count[c] == kBtCount[c], FSI_E_ARG, "unexpected B^T stencil width");
    for (int k = 0; k < t64.bt_count[c]; ++k) {
      FSI_REQUIRE(t64.bt_off[c][k][0] == dofs.bt[c][k][0] && t64.bt_off[c][k][1] == dofs.bt[c][k][1], FSI_E_ARG,
                  "B^T offsets differ from the compiled pattern");
      t32.bt_off[c][k][0] = t64.bt_off[c][k][0];
      t32.bt_off[c][k][1] = t64.bt_off[c][k][1];
    }
  }
  sort_entries(t64.b_count, t64.b_off, t64.b_coef, t64.b_lds);
  FSI_REQUIRE(t64.b_count == kStencilCount[0], FSI_E_ARG, "unexpected B stencil width");
  for (int k = 0; k < t64.b_count; ++k) {
    FSI_REQUIRE(t64.b_off[k][0] == sofs.d[0][k][0] && t64.b_off[k][1] == sofs.d[0][k][1], FSI_E_ARG,
                "B offsets differ from the compiled pattern");
    t32.b_off[k][0] = t64.b_off[k][0];
    t32.b_off[k][1] = t64.b_off[k][1];
    t32.b_lds[k] = t64.b_lds[k];
  }
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < kBtMax; ++k)
      for (int al = 0; al < 2; ++al) t32.bt_coef[c][k][al] = (float)t64.bt_coef[c][k][al];
  for (int k = 0; k < kBMax; ++k)
    for (int al = 0; al < 2; ++al) t32.b_coef[k][al] = (float)t64.b_coef[k][al];
}

// Host: rows of a P1 x P1 matrix (EM_MP: mass, EM_LP: Laplacian) at one node of each of
// the nine position classes of an n x n grid, summed over the triangles around the node.
void p1_tables(int n, int which, int pin, P1Table<double> &t64, P1Table<float> &t32) {
  FSI_REQUIRE(n >= 2, FSI_E_ARG, "P1 tables need n >= 2");
  std::vector<double> E;
  element_tables(n, 1.0, E);
  std::memset(&t64, 0, sizeof(t64));
  std::memset(&t32, 0, sizeof(t32));
  static const int nb[kP1Nbr][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, 1}};
  const int rep[3] = {0, 1, n};
  for (int cls = 0; cls < 9; ++cls) {
    const int i = rep[cls % 3], j = rep[cls / 3];
    for (int k = 0; k < kP1Nbr; ++k) {
      const int i2 = i + nb[k][0], j2 = j + nb[k][1];
      double v = 0.0;
      for (int cj = std::max(0, j - 1); cj <= std::min(n - 1, j); ++cj)
        for (int ci = std::max(0, i - 1); ci <= std::min(n - 1, i); ++ci)
          for (int t = 0; t < 2; ++t) {
            int a = -1, b = -1;
            for (int q = 0; q < 3; ++q) {
              if (2 * ci + hOff[t][q][0] == 2 * i && 2 * cj + hOff[t][q][1] == 2 * j) a = q;
              if (2 * ci + hOff[t][q][0] == 2 * i2 && 2 * cj + hOff[t][q][1] == 2 * j2) b = q;
            }
            if (a >= 0 && b >= 0) v += E[t * EM_SIZE + which + a * 3 + b];
          }
      if (pin && cls == 0) v = (k == 0) ? 1.0 : 0.0;   // identity row of the pinned node 0
      t64.coef[cls][k] = v;
      t32.coef[cls][k] = (float)v;
    }
    FSI_REQUIRE(t64.coef[cls][0] > 0.0, FSI_E_ARG, "P1 table: non-positive diagonal");
    t64.dinv[cls] = 1.0 / t64.coef[cls][0];
    t32.dinv[cls] = (float)t64.dinv[cls];
  }
  t64.pin = t32.pin = pin;
}

// ---------------------------------------------------------------- structured adjacency
struct Adj {
  int ci, cj, t, a;
};

// Triangles containing P2 lattice node (I, J) (0 <= I, J <= 2n), with the node's local
// index a in each.  At most 6 (out must hold 8).
__device__ __forceinline__ int adjacent_tris(int I, int J, int n, Adj *out) {
  int ilo = (I - 1) >> 1, ihi = I >> 1, jlo = (J - 1) >> 1, jhi = J >> 1;
  if (ilo < 0) ilo = 0;
  if (jlo < 0) jlo = 0;
  if (ihi > n - 1) ihi = n - 1;
  if (jhi > n - 1) jhi = n - 1;
  int cnt = 0;
  for (int cj = jlo; cj <= jhi; ++cj)
    for (int ci = ilo; ci <= ihi; ++ci)
      for (int t = 0; t < 2; ++t)
        for (int a = 0; a < 6; ++a)
          if (2 * ci + kOff[t][a][0] == I && 2 * cj + kOff[t][a][1] == J) {
            out[cnt++] = Adj{ci, cj, t, a};
            break;
          }
  return cnt;
}

__device__ __forceinline__ int local_of(const Adj &t, int I, int J) {
  for (int b = 0; b < 6; ++b)
    if (2 * t.ci + kOff[t.t][b][0] == I && 2 * t.cj + kOff[t.t][b][1] == J) return b;
  return -1;
}

__device__ __forceinline__ bool p2_boundary(int I, int J, int n) {
  return I == 0 || J == 0 || I == 2 * n || J == 2 * n;
}

// P2 x P2 rows: A_f (width 4, BC by value) and optionally M_f (width 1, no BC).
// pass 0: cnt[row] = number of columns; pass 1: fill.
__global__ void k_asm_p2p2(int n, int pass, const double *__restrict__ E, double rdt,
                           int *cnt, const int *rowptr, int *col, double *A, double *M) {
  int64_t L = 2 * n + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  int I = (int)(row % L), J = (int)(row / L);
  Adj adj[8];
  int na = adjacent_tris(I, J, n, adj);
  bool rb = p2_boundary(I, J, n);
  int k = pass ? rowptr[row] : 0;
  int c = 0;
  for (int dJ = -2; dJ <= 2; ++dJ)
    for (int dI = -2; dI <= 2; ++dI) {
      int I2 = I + dI, J2 = J + dJ;
      if (I2 < 0 || J2 < 0 || I2 > 2 * n || J2 > 2 * n) continue;
      bool touched = false;
      double m = 0, kxx = 0, kxy = 0, kyx = 0, kyy = 0;
      for (int q = 0; q < na; ++q) {
        int b = local_of(adj[q], I2, J2);
        if (b < 0) continue;
        touched = true;
        const double *e = E + adj[q].t * EM_SIZE;
        int a = adj[q].a;
        m += e[EM_M + a * 6 + b];
        kxx += e[EM_K + ((0 * 2 + 0) * 6 + a) * 6 + b];
        kxy += e[EM_K + ((0 * 2 + 1) * 6 + a) * 6 + b];
        kyx += e[EM_K + ((1 * 2 + 0) * 6 + a) * 6 + b];
        kyy += e[EM_K + ((1 * 2 + 1) * 6 + a) * 6 + b];
      }
      if (!touched) continue;
      if (pass) {
        int64_t cidx = (int64_t)J2 * L + I2;
        col[k] = (int)cidx;
        double *v = A + 4 * (int64_t)k;
        if (rb || p2_boundary(I2, J2, n)) {
          double dg = (cidx == row) ? 1.0 : 0.0;
          v[0] = dg; v[1] = 0.0; v[2] = 0.0; v[3] = dg;
        } else {
          v[0] = rdt * m + kxx; v[1] = kxy; v[2] = kyx; v[3] = rdt * m + kyy;
        }
        if (M) M[k] = m;
        ++k;
      }
      ++c;
    }
  if (!pass) cnt[row] = c;
}

// Rows of B (P1 node (i, j)), columns P2 nodes; width 2; row 0 and boundary columns zero.
__global__ void k_asm_b(int n, int pass, const double *__restrict__ E, int *cnt,
                        const int *rowptr, int *col, double *V) {
  int64_t L1 = n + 1, L = 2 * n + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L1 * L1) return;
  int I = 2 * (int)(row % L1), J = 2 * (int)(row / L1);
  Adj adj[8];
  int na = adjacent_tris(I, J, n, adj);
  int k = pass ? rowptr[row] : 0, c = 0;
  for (int dJ = -2; dJ <= 2; ++dJ)
    for (int dI = -2; dI <= 2; ++dI) {
      int I2 = I + dI, J2 = J + dJ;
      if (I2 < 0 || J2 < 0 || I2 > 2 * n || J2 > 2 * n) continue;
      bool touched = false;
      double bx = 0, by = 0;
      for (int q = 0; q < na; ++q) {
        int b = local_of(adj[q], I2, J2);
        if (b < 0) continue;
        touched = true;
        const double *e = E + adj[q].t * EM_SIZE;
        int a = adj[q].a;   // vertex: P1 local index = P2 local index
        bx += e[EM_B + (0 * 3 + a) * 6 + b];
        by += e[EM_B + (1 * 3 + a) * 6 + b];
      }
      if (!touched) continue;
      if (pass) {
        col[k] = (int)((int64_t)J2 * L + I2);
        bool z = (row == 0) || p2_boundary(I2, J2, n);
        V[2 * (int64_t)k] = z ? 0.0 : bx;
        V[2 * (int64_t)k + 1] = z ? 0.0 : by;
        ++k;
      }
      ++c;
    }
  if (!pass) cnt[row] = c;
}

// Rows of B^T (P2 node (I, J)), columns P1 nodes; width 2; boundary rows and column 0 zero.
__global__ void k_asm_bt(int n, int pass, const double *__restrict__ E, int *cnt,
                         const int *rowptr, int *col, double *V) {
  int64_t L = 2 * n + 1, L1 = n + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  int I = (int)(row % L), J = (int)(row / L);
  Adj adj[8];
  int na = adjacent_tris(I, J, n, adj);
  bool rb = p2_boundary(I, J, n);
  int ilo = (I - 1) >> 1, ihi = (I + 2) >> 1, jlo = (J - 1) >> 1, jhi = (J + 2) >> 1;
  if (ilo < 0) ilo = 0;
  if (jlo < 0) jlo = 0;
  if (ihi > n) ihi = n;
  if (jhi > n) jhi = n;
  int k = pass ? rowptr[row] : 0, c = 0;
  for (int j2 = jlo; j2 <= jhi; ++j2)
    for (int i2 = ilo; i2 <= ihi; ++i2) {
      bool touched = false;
      double bx = 0, by = 0;
      for (int q = 0; q < na; ++q) {
        int b = local_of(adj[q], 2 * i2, 2 * j2);
        if (b < 0) continue;      // b in {0, 1, 2}: a vertex of the triangle
        touched = true;
        const double *e = E + adj[q].t * EM_SIZE;
        int a = adj[q].a;
        bx += e[EM_B + (0 * 3 + b) * 6 + a];
        by += e[EM_B + (1 * 3 + b) * 6 + a];
      }
      if (!touched) continue;
      if (pass) {
        int64_t cidx = (int64_t)j2 * L1 + i2;
        col[k] = (int)cidx;
        bool z = rb || cidx == 0;
        V[2 * (int64_t)k] = z ? 0.0 : bx;
        V[2 * (int64_t)k + 1] = z ? 0.0 : by;
        ++k;
      }
      ++c;
    }
  if (!pass) cnt[row] = c;
}

// P1 x P1 rows (P1 node (i, j)) of the table entry `which` (EM_MP or EM_LP); with `pin`
// row and column 0 are zeroed and (0, 0) = 1.
__global__ void k_asm_p1p1(int n, int pass, const double *__restrict__ E, int which, int pin,
                           int *cnt, const int *rowptr, int *col, double *V) {
  int64_t L1 = n + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L1 * L1) return;
  int i = (int)(row % L1), j = (int)(row / L1);
  Adj adj[8];
  int na = adjacent_tris(2 * i, 2 * j, n, adj);
  int k = pass ? rowptr[row] : 0, c = 0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      int i2 = i + di, j2 = j + dj;
      if (i2 < 0 || j2 < 0 || i2 > n || j2 > n) continue;
      bool touched = false;
      double v = 0;
      for (int q = 0; q < na; ++q) {
        int b = local_of(adj[q], 2 * i2, 2 * j2);
        if (b < 0) continue;
        touched = true;
        v += E[adj[q].t * EM_SIZE + which + adj[q].a * 3 + b];
      }
      if (!touched) continue;
      if (pass) {
        int64_t cidx = (int64_t)j2 * L1 + i2;
        col[k] = (int)cidx;
        if (pin && (row == 0 || cidx == 0)) v = (row == cidx) ? 1.0 : 0.0;
        V[k] = v;
        ++k;
      }
      ++c;
    }
  if (!pass) cnt[row] = c;
}

__global__ void k_p2_boundary_flags(int n, unsigned char *bnd) {
  int64_t L = 2 * n + 1;
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= L * L) return;
  bnd[r] = p2_boundary((int)(r % L), (int)(r / L), n) ? 1 : 0;
}

// Two-pass row builder shared by every structured block.
template <typename Launch>
static void build_rows(Csr &A, int64_t nrows, int64_t ncols, int width, hipStream_t s,
                       DevBuf<int> &tmp, Launch launch, bool with_m = false,
                       DevBuf<double> *M = nullptr) {
  A.nrows = nrows;
  A.ncols = ncols;
  A.width = width;
  A.rowptr.alloc(nrows + 1);
  launch(0, A.rowptr.p, nullptr, nullptr, nullptr, nullptr);
  scan_excl(A.rowptr.p, A.rowptr.p, nrows, tmp, s);
  int nnz = 0;
  FSI_HIP(hipMemcpyAsync(&nnz, A.rowptr.p + nrows, sizeof(int), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  A.nnz = nnz;
  A.col.alloc(nnz);
  A.val.alloc((size_t)nnz * width);
  if (with_m) M->alloc(nnz);
  launch(1, nullptr, A.rowptr.p, A.col.p, A.val.p, with_m ? M->p : nullptr);
  FSI_CHECK_LAUNCH();
}

static void assemble_p2p2(Csr &A, DevBuf<double> *M, int n, const double *dE, double rdt,
                          DevBuf<int> &tmp, hipStream_t s) {
  int64_t rows = (int64_t)(2 * n + 1) * (2 * n + 1);
  unsigned g = grid_for(rows, 256);
  build_rows(A, rows, rows, 4, s, tmp,
             [&](int pass, int *cnt, const int *rp, int *col, double *v, double *m) {
               hipLaunchKernelGGL(k_asm_p2p2, dim3(g), dim3(256), 0, s, n, pass, dE, rdt, cnt,
                                  rp, col, v, m);
             },
             M != nullptr, M);
}

static void assemble_p1p1(Csr &A, int n, const double *dE, int which, int pin, DevBuf<int> &tmp,
                          hipStream_t s) {
  int64_t rows = (int64_t)(n + 1) * (n + 1);
  unsigned g = grid_for(rows, 256);
  build_rows(A, rows, rows, 1, s, tmp,
             [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
               hipLaunchKernelGGL(k_asm_p1p1, dim3(g), dim3(256), 0, s, n, pass, dE, which, pin,
                                  cnt, rp, col, v);
             });
}

void build_fluid(Ctx &c) {
  hipStream_t s = c.stream;
  std::vector<double> hE;
  element_tables(c.n, c.nu, hE);
  DevBuf<double> dE(hE.size());
  FSI_HIP(hipMemcpyAsync(dE.p, hE.data(), hE.size() * sizeof(double), hipMemcpyHostToDevice, s));
  DevBuf<int> tmp;
  const int n = c.n;
  assemble_p2p2(c.Af, &c.Mf, n, dE.p, c.rho / c.dt, tmp, s);
  int64_t np = (int64_t)(n + 1) * (n + 1), n2 = (int64_t)(2 * n + 1) * (2 * n + 1);
  unsigned gp = grid_for(np, 256), g2 = grid_for(n2, 256);
  build_rows(c.B, np, n2, 2, s, tmp,
             [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
               hipLaunchKernelGGL(k_asm_b, dim3(gp), dim3(256), 0, s, n, pass, dE.p, cnt, rp, col, v);
             });
  build_rows(c.BT, n2, np, 2, s, tmp,
             [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
               hipLaunchKernelGGL(k_asm_bt, dim3(g2), dim3(256), 0, s, n, pass, dE.p, cnt, rp, col, v);
             });
  assemble_p1p1(c.Mp, n, dE.p, EM_MP, 0, tmp, s);
  c.Mp_dinv.alloc(np);
  hipLaunchKernelGGL(k_diag_inv, dim3(gp), dim3(256), 0, s, np, c.Mp.rowptr.p, c.Mp.col.p, c.Mp.val.p,
                     c.Mp_dinv.p);
  {
    DivTable<double> t64;
    DivTable<float> t32;
    div_tables(n, t64, t32);
    upload_bytes(c.divtab64, &t64, sizeof(t64), s);
    upload_bytes(c.divtab32, &t32, sizeof(t32), s);
  }
  {
    P1Table<double> t64;
    P1Table<float> t32;
    p1_tables(n, EM_MP, 0, t64, t32);
    upload_bytes(c.mptab64, &t64, sizeof(t64), s);
    upload_bytes(c.mptab32, &t32, sizeof(t32), s);
  }
  c.bnd.alloc(n2);
  hipLaunchKernelGGL(k_p2_boundary_flags, dim3(g2), dim3(256), 0, s, n, c.bnd.p);
  FSI_CHECK_LAUNCH();
  FSI_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- solid blocks
// Row l gathers, over the triangles around node l (sorted by element id), the P1
// stiffness kappa |E| grad l_a . grad l_b and mass |E| (1 + delta_ab) / 12.
__global__ void k_asm_solid(int64_t ns, const int *__restrict__ n2e_ptr, const int *__restrict__ n2e,
                            const int *__restrict__ tri, const double *__restrict__ xy,
                            const int *__restrict__ rowptr, const int *__restrict__ col,
                            double kappa, double *As, double *Cs) {
  int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ns) return;
  int r0 = rowptr[l], r1 = rowptr[l + 1];
  for (int k = r0; k < r1; ++k) { As[k] = 0.0; Cs[k] = 0.0; }
  for (int q = n2e_ptr[l]; q < n2e_ptr[l + 1]; ++q) {
    int e = n2e[q] >> 2, a = n2e[q] & 3;
    int v[3] = {tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]};
    double x[3], y[3];
    for (int m = 0; m < 3; ++m) { x[m] = xy[v[m]]; y[m] = xy[ns + v[m]]; }
    double d = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    double area = 0.5 * d;
    double gx[3] = {(y[1] - y[2]) / d, (y[2] - y[0]) / d, (y[0] - y[1]) / d};
    double gy[3] = {(x[2] - x[1]) / d, (x[0] - x[2]) / d, (x[1] - x[0]) / d};
    for (int b = 0; b < 3; ++b) {
      int cb = v[b];
      int pos = r0;
      while (pos < r1 && col[pos] != cb) ++pos;
      As[pos] += kappa * area * (gx[a] * gx[b] + gy[a] * gy[b]);
      Cs[pos] += area * (a == b ? 2.0 : 1.0) / 12.0;
    }
  }
}

// Q1: row l gathers over the quadrilaterals around node l (sorted by element id) kappa
// (grad N_a, grad N_b) and (N_a, N_b) by the 2 x 2 Gauss rule in (xi, eta) on the bilinear map
// of the reference element (exact on parallelograms).
__global__ void k_asm_q1(int64_t ns, const int *__restrict__ n2e_ptr, const int *__restrict__ n2e,
                         const int *__restrict__ quad, const double *__restrict__ xy, const int *__restrict__ rowptr,
                         const int *__restrict__ col, double kappa, double *As, double *Cs) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ns) return;
  const int r0 = rowptr[l], r1 = rowptr[l + 1];
  for (int k = r0; k < r1; ++k) { As[k] = 0.0; Cs[k] = 0.0; }
  const double g[2] = {0.5 - 0.5 / 1.7320508075688772, 0.5 + 0.5 / 1.7320508075688772};
  for (int q = n2e_ptr[l]; q < n2e_ptr[l + 1]; ++q) {
    const int e = n2e[q] >> 2, a = n2e[q] & 3;
    int v[4];
    double x[4], y[4];
    for (int m = 0; m < 4; ++m) {
      v[m] = quad[4 * e + m];
      x[m] = xy[v[m]];
      y[m] = xy[ns + v[m]];
    }
    double ka[4] = {0, 0, 0, 0}, ma[4] = {0, 0, 0, 0};
    for (int pq = 0; pq < 4; ++pq) {
      const double xi = g[pq & 1], eta = g[pq >> 1];
      const double N[4] = {(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta};
      const double Nx[4] = {-(1 - eta), 1 - eta, eta, -eta};
      const double Ne[4] = {-(1 - xi), -xi, xi, 1 - xi};
      double j00 = 0, j01 = 0, j10 = 0, j11 = 0;
      for (int m = 0; m < 4; ++m) {
        j00 += Nx[m] * x[m];
        j01 += Ne[m] * x[m];
        j10 += Nx[m] * y[m];
        j11 += Ne[m] * y[m];
      }
      const double det = j00 * j11 - j01 * j10;
      double gx[4], gy[4];
      for (int m = 0; m < 4; ++m) {
        gx[m] = (j11 * Nx[m] - j10 * Ne[m]) / det;
        gy[m] = (j00 * Ne[m] - j01 * Nx[m]) / det;
      }
      const double wt = 0.25 * det;
      for (int b = 0; b < 4; ++b) {
        ka[b] += wt * (gx[a] * gx[b] + gy[a] * gy[b]);
        ma[b] += wt * N[a] * N[b];
      }
    }
    for (int b = 0; b < 4; ++b) {
      int pos = r0;
      while (pos < r1 && col[pos] != v[b]) ++pos;
      As[pos] += kappa * ka[b];
      Cs[pos] += ma[b];
    }
  }
}

// the transposed copy of the solid pattern and its two value arrays (one thread per row)
__global__ void k_solid_ell(int64_t ns, int w, const int *rp, const int *col, const double *as, const double *cs,
                            int *ecol, double *eas, double *ecs) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ns) return;
  const int k0 = rp[r], k1 = rp[r + 1];
  for (int u = 0; u < w; ++u) {
    const bool in = k0 + u < k1;
    ecol[(int64_t)u * ns + r] = in ? col[k0 + u] : (int)r;
    eas[(int64_t)u * ns + r] = in ? as[k0 + u] : 0.0;
    ecs[(int64_t)u * ns + r] = in ? cs[k0 + u] : 0.0;
  }
}

__global__ void k_diag_inv(int64_t nrows, const int *rowptr, const int *col, const double *v,
                           double *dinv) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  double d = 0.0;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k)
    if (col[k] == r) d = v[k];
  dinv[r] = 1.0 / d;
}

void build_solid(Ctx &c) {
  hipStream_t s = c.stream;
  const int64_t ns = c.Ns, nt = c.Nt;
  const bool quads = c.pair == FSI_PAIR_Q2P1DISC;
  const int nv = quads ? 4 : 3;   // vertices per element
  // reference areas (validated on the host: counter-clockwise, non-degenerate; a
  // quadrilateral strictly convex)
  std::vector<double> area(nt);
  for (int64_t e = 0; e < nt; ++e) {
    const int *t = &c.h_tri[nv * e];
    for (int m = 0; m < nv; ++m)
      FSI_REQUIRE(t[m] >= 0 && t[m] < ns, FSI_E_ARG, "solid element refers to a missing node");
    double a = 0.0;
    bool convex = true;
    for (int m = 0; m < nv; ++m) {
      const int p = t[(m + nv - 1) % nv], q = t[m], r = t[(m + 1) % nv];
      a += c.h_xy[q] * c.h_xy[ns + r] - c.h_xy[r] * c.h_xy[ns + q];
      const double cr = (c.h_xy[q] - c.h_xy[p]) * (c.h_xy[ns + r] - c.h_xy[ns + q]) -
                        (c.h_xy[ns + q] - c.h_xy[ns + p]) * (c.h_xy[r] - c.h_xy[q]);
      convex = convex && cr > 0.0;
    }
    area[e] = 0.5 * a;
    if (!quads) {   // the triangle's area as the coupling uses it
      double x0 = c.h_xy[t[0]], y0 = c.h_xy[ns + t[0]];
      double x1 = c.h_xy[t[1]], y1 = c.h_xy[ns + t[1]];
      double x2 = c.h_xy[t[2]], y2 = c.h_xy[ns + t[2]];
      area[e] = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
      convex = area[e] > 0.0;
    }
    FSI_REQUIRE(area[e] > 0.0 && convex, FSI_E_MESH,
                "solid reference element " + std::to_string(e) + " is degenerate, clockwise or not convex");
  }
  // node -> (element, local vertex), sorted by element
  std::vector<int> cnt(ns + 1, 0);
  for (int64_t e = 0; e < nt; ++e)
    for (int m = 0; m < nv; ++m) cnt[c.h_tri[nv * e + m] + 1]++;
  for (int64_t l = 0; l < ns; ++l) cnt[l + 1] += cnt[l];
  std::vector<int> adj(cnt[ns]);
  std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
  c.max_adj = 0;
  for (int64_t e = 0; e < nt; ++e)
    for (int m = 0; m < nv; ++m) adj[fillp[c.h_tri[nv * e + m]]++] = (int)(4 * e + m);
  for (int64_t l = 0; l < ns; ++l) {
    c.max_adj = std::max(c.max_adj, cnt[l + 1] - cnt[l]);
    FSI_REQUIRE(cnt[l + 1] > cnt[l], FSI_E_MESH, "solid node " + std::to_string(l) + " is in no element");
  }
  FSI_REQUIRE(4 * nt < (int64_t)INT32_MAX, FSI_E_ARG, "too many solid elements");
  // pattern: sorted unique neighbours
  std::vector<int> rp(ns + 1, 0), cols;
  cols.reserve(7 * ns);
  std::vector<int> tmpn;
  for (int64_t l = 0; l < ns; ++l) {
    tmpn.clear();
    for (int q = cnt[l]; q < cnt[l + 1]; ++q) {
      int e = adj[q] >> 2;
      for (int m = 0; m < nv; ++m) tmpn.push_back(c.h_tri[nv * e + m]);
    }
    std::sort(tmpn.begin(), tmpn.end());
    tmpn.erase(std::unique(tmpn.begin(), tmpn.end()), tmpn.end());
    cols.insert(cols.end(), tmpn.begin(), tmpn.end());
    rp[l + 1] = (int)cols.size();
  }
  // grow-only buffers: a context re-meshed with a solid of equal or smaller size
  // (fsi_set_solid) allocates nothing
  auto up = [&](auto &buf, const auto &vec) {
    using T = typename std::decay_t<decltype(vec)>::value_type;
    buf.reserve(vec.size());
    FSI_HIP(hipMemcpyAsync(buf.p, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, s));
  };
  up(c.tri, c.h_tri);
  up(c.ref_xy, c.h_xy);
  up(c.ref_area, area);
  up(c.n2e_ptr, cnt);
  up(c.n2e, adj);
  c.S.nrows = ns; c.S.ncols = ns; c.S.width = 1; c.S.nnz = (int64_t)cols.size();
  up(c.S.rowptr, rp);
  up(c.S.col, cols);
  c.S.val.reserve(cols.size());
  c.Cs.reserve(cols.size());
  if (quads)
    hipLaunchKernelGGL(k_asm_q1, dim3(grid_for(ns, 256)), dim3(256), 0, s, ns, c.n2e_ptr.p, c.n2e.p, c.tri.p,
                       c.ref_xy.p, c.S.rowptr.p, c.S.col.p, c.kappa, c.S.val.p, c.Cs.p);
  else
    hipLaunchKernelGGL(k_asm_solid, dim3(grid_for(ns, 256)), dim3(256), 0, s, ns, c.n2e_ptr.p,
                       c.n2e.p, c.tri.p, c.ref_xy.p, c.S.rowptr.p, c.S.col.p, c.kappa, c.S.val.p,
                       c.Cs.p);
  c.Cs_dinv.reserve(ns);
  hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(ns, 256)), dim3(256), 0, s, ns, c.S.rowptr.p,
                     c.S.col.p, c.Cs.p, c.Cs_dinv.p);
  int ew = 1;
  for (int64_t l = 0; l < ns; ++l) ew = std::max(ew, rp[l + 1] - rp[l]);
  c.s_ew = ew;
  c.s_ecol.reserve((size_t)ew * ns);
  c.s_eas.reserve((size_t)ew * ns);
  c.s_ecs.reserve((size_t)ew * ns);
  hipLaunchKernelGGL(k_solid_ell, dim3(grid_for(ns, 256)), dim3(256), 0, s, ns, ew, c.S.rowptr.p, c.S.col.p,
                     c.S.val.p, c.Cs.p, c.s_ecol.p, c.s_eas.p, c.s_ecs.p);
  FSI_CHECK_LAUNCH();
  c.Cs32.reserve(cols.size());
  convert(c.Cs32.p, c.Cs.p, (int64_t)cols.size(), s);
  c.Cs_dinv32.reserve(ns);
  convert(c.Cs_dinv32.p, c.Cs_dinv.p, ns, s);
  FSI_HIP(hipStreamSynchronize(s));
  if (quads) {
    // Chebyshev interval of D^{-1} C_s: [1/4, 9/4] on rectangles (the tensor product of the 1D
    // [1/2, 3/2]); the upper end raised to the Gershgorin bound max_l sum_m |C_lm| / C_ll where
    // a mesh exceeds it
    std::vector<double> hc(cols.size());
    FSI_HIP(hipMemcpy(hc.data(), c.Cs.p, hc.size() * sizeof(double), hipMemcpyDeviceToHost));
    double g = 0.0;
    for (int64_t l = 0; l < ns; ++l) {
      double d = 0.0, sum = 0.0;
      for (int k = rp[l]; k < rp[l + 1]; ++k) {
        sum += std::fabs(hc[k]);
        if (cols[k] == l) d = hc[k];
      }
      FSI_REQUIRE(d > 0.0, FSI_E_MESH, "solid mass with a non-positive diagonal");
      g = std::max(g, sum / d);
    }
    c.cs_lo = 0.25;
    c.cs_hi = std::max(2.25, g);
    c.cs_nsteps = 56;   // (1 - 1/3)/(1 + 1/3) = 1/2 per step on [1/4, 9/4]: 2^-56 < 1e-16
  } else {
    c.cs_lo = 0.5;
    c.cs_hi = 2.0;
    c.cs_nsteps = 36;
  }
}

// ---------------------------------------------------------------- multigrid transfers
// Coarse P2 weights at fine P2 lattice node (I, J) of an nf grid (coarse grid nf / 2):
// the fine node lies in a coarse triangle where the coarse quadratic basis is evaluated
// exactly (barycentric coordinates are multiples of 1/4).  Returns the entries with
// non-zero weight at interior coarse nodes, sorted by coarse index.
__device__ int p2_prolong_row(int I, int J, int nf, int *cidx, double *w) {
  int nc = nf / 2;
  int64_t Lc = 2 * nc + 1;
  int ci = I / 4, cj = J / 4;
  if (ci > nc - 1) ci = nc - 1;
  if (cj > nc - 1) cj = nc - 1;
  double xi = (I - 4 * ci) * 0.25, eta = (J - 4 * cj) * 0.25;
  int t;
  double l[3];
  if (xi >= eta) { t = 0; l[0] = 1.0 - xi; l[1] = xi - eta; l[2] = eta; }
  else { t = 1; l[0] = 1.0 - eta; l[1] = xi; l[2] = eta - xi; }
  double phi[6] = {l[0] * (2 * l[0] - 1), l[1] * (2 * l[1] - 1), l[2] * (2 * l[2] - 1),
                   4 * l[0] * l[1], 4 * l[1] * l[2], 4 * l[2] * l[0]};
  int cnt = 0;
  for (int b = 0; b < 6; ++b) {
    if (phi[b] == 0.0) continue;
    int Ic = 2 * ci + kOff[t][b][0], Jc = 2 * cj + kOff[t][b][1];
    if (Ic == 0 || Jc == 0 || Ic == 2 * nc || Jc == 2 * nc) continue;
    int idx = (int)(Jc * Lc + Ic);
    int p = cnt++;
    while (p > 0 && cidx[p - 1] > idx) { cidx[p] = cidx[p - 1]; w[p] = w[p - 1]; --p; }
    cidx[p] = idx;
    w[p] = phi[b];
  }
  return cnt;
}

__global__ void k_p2_prolong(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  int64_t L = 2 * nf + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  int I = (int)(row % L), J = (int)(row / L);
  int ci[6];
  double w[6];
  int m = p2_boundary(I, J, nf) ? 0 : p2_prolong_row(I, J, nf, ci, w);
  if (!pass) { cnt[row] = m; return; }
  int k = rowptr[row];
  for (int q = 0; q < m; ++q) { col[k + q] = ci[q]; V[k + q] = w[q]; }
}

__global__ void k_p2_restrict(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  int nc = nf / 2;
  int64_t Lc = 2 * nc + 1, L = 2 * nf + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Lc * Lc) return;
  int Ic = (int)(row % Lc), Jc = (int)(row / Lc);
  int k = pass ? rowptr[row] : 0, c = 0;
  if (!p2_boundary(Ic, Jc, nc)) {
    for (int J = 2 * Jc - 4; J <= 2 * Jc + 4; ++J)
      for (int I = 2 * Ic - 4; I <= 2 * Ic + 4; ++I) {
        if (I < 0 || J < 0 || I > 2 * nf || J > 2 * nf || p2_boundary(I, J, nf)) continue;
        int ci[6];
        double w[6];
        int m = p2_prolong_row(I, J, nf, ci, w);
        for (int q = 0; q < m; ++q)
          if (ci[q] == row) {
            if (pass) { col[k] = (int)((int64_t)J * L + I); V[k] = w[q]; ++k; }
            ++c;
          }
      }
  }
  if (!pass) cnt[row] = c;
}

// P1 (pressure) prolongation: linear interpolation on the nested triangulation; fine
// node 0 and coarse node 0 (the pinned pressure node) are excluded.
__device__ int p1_prolong_row(int i, int j, int nf, int *cidx, double *w) {
  int nc = nf / 2;
  int64_t Lc = nc + 1;
  int ci = i >> 1, cj = j >> 1;
  int pts[2][2];
  int m;
  if (!(i & 1) && !(j & 1)) { pts[0][0] = ci; pts[0][1] = cj; m = 1; }
  else if ((i & 1) && !(j & 1)) { pts[0][0] = ci; pts[0][1] = cj; pts[1][0] = ci + 1; pts[1][1] = cj; m = 2; }
  else if (!(i & 1) && (j & 1)) { pts[0][0] = ci; pts[0][1] = cj; pts[1][0] = ci; pts[1][1] = cj + 1; m = 2; }
  else { pts[0][0] = ci; pts[0][1] = cj; pts[1][0] = ci + 1; pts[1][1] = cj + 1; m = 2; }
  int cnt = 0;
  for (int q = 0; q < m; ++q) {
    int idx = (int)(pts[q][1] * Lc + pts[q][0]);
    if (idx == 0) continue;
    cidx[cnt] = idx;
    w[cnt] = (m == 1) ? 1.0 : 0.5;
    ++cnt;
  }
  return cnt;
}

__global__ void k_p1_prolong(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  int64_t L = nf + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  int ci[2];
  double w[2];
  int m = row == 0 ? 0 : p1_prolong_row((int)(row % L), (int)(row / L), nf, ci, w);
  if (!pass) { cnt[row] = m; return; }
  int k = rowptr[row];
  for (int q = 0; q < m; ++q) { col[k + q] = ci[q]; V[k + q] = w[q]; }
}

__global__ void k_p1_restrict(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  int nc = nf / 2;
  int64_t Lc = nc + 1, L = nf + 1;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Lc * Lc) return;
  int ic = (int)(row % Lc), jc = (int)(row / Lc);
  int k = pass ? rowptr[row] : 0, c = 0;
  if (row != 0) {
    for (int j = 2 * jc - 1; j <= 2 * jc + 1; ++j)
      for (int i = 2 * ic - 1; i <= 2 * ic + 1; ++i) {
        if (i < 0 || j < 0 || i > nf || j > nf) continue;
        int64_t f = (int64_t)j * L + i;
        if (f == 0) continue;
        int cidx[2];
        double w[2];
        int m = p1_prolong_row(i, j, nf, cidx, w);
        for (int q = 0; q < m; ++q)
          if (cidx[q] == row) {
            if (pass) { col[k] = (int)f; V[k] = w[q]; ++k; }
            ++c;
          }
      }
  }
  if (!pass) cnt[row] = c;
}

// Inverse of the 2x2 diagonal blocks (width 4) or of the scalar diagonal (width 1).
__global__ void k_block_diag_inv(int64_t nrows, int width, const int *rowptr, const int *col,
                                 const double *v, double *dinv) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    if (col[k] != r) continue;
    if (width == 4) {
      double a = v[4 * (int64_t)k], b = v[4 * (int64_t)k + 1], c = v[4 * (int64_t)k + 2],
             d = v[4 * (int64_t)k + 3];
      double det = a * d - b * c;
      dinv[4 * r] = d / det;
      dinv[4 * r + 1] = -b / det;
      dinv[4 * r + 2] = -c / det;
      dinv[4 * r + 3] = a / det;
    } else {
      dinv[r] = 1.0 / v[k];
    }
  }
}

// z = Dinv y (2x2 blocks: NC = 2, stride nodes; scalar: NC = 1)
__global__ void k_apply_dinv(int64_t nodes, int width, const double *dinv, const double *y,
                             double *z) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nodes) return;
  if (width == 4) {
    double a = y[r], b = y[nodes + r];
    z[r] = dinv[4 * r] * a + dinv[4 * r + 1] * b;
    z[nodes + r] = dinv[4 * r + 2] * a + dinv[4 * r + 3] * b;
  } else {
    z[r] = dinv[r] * y[r];
  }
}

static double dev_norm(const double *d, int64_t n, DevBuf<double> &part, DevBuf<double> &out,
                       hipStream_t s) {
  multidot(d, 0, 1, d, n, out.p, part, s);
  double h = 0.0;
  FSI_HIP(hipMemcpyAsync(&h, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  return std::sqrt(h);
}

// lambda_max(D^{-1} A) by power iteration from a fixed pseudo-random start.
static double power_lmax(MgLevel &L, int comps, hipStream_t s) {
  int64_t m = comps * L.nodes;
  std::vector<double> h(m);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (int64_t i = 0; i < m; ++i) {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    h[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  DevBuf<double> x(m), y(m), part, out(1);
  FSI_HIP(hipMemcpyAsync(x.p, h.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
  double lam = 0.0, nx = dev_norm(x.p, m, part, out, s);
  for (int it = 0; it < 30; ++it) {
    if (L.A.width == 4)
      spmv<double, 4, 2, SP_APPLY>(L.A.nrows, L.A.rowptr.p, L.A.col.p, L.A.val.p, x.p, L.nodes,
                                   y.p, L.nodes, s);
    else
      spmv<double, 1, 1, SP_APPLY>(L.A.nrows, L.A.rowptr.p, L.A.col.p, L.A.val.p, x.p, L.nodes,
                                   y.p, L.nodes, s);
    hipLaunchKernelGGL(k_apply_dinv, dim3(grid_for(L.nodes, 256)), dim3(256), 0, s, L.nodes,
                       L.A.width, L.dinv.p, y.p, x.p);
    FSI_CHECK_LAUNCH();
    double nz = dev_norm(x.p, m, part, out, s);
    lam = nz / nx;
    axpby(x.p, x.p, 1.0 / nz, 0.0, m, s);
    nx = 1.0;
  }
  return lam;
}

// Dense inverse of the coarsest operator by Gauss-Jordan elimination with partial
// pivoting (host, FP64).  Unknown order: component-major ([x | y] for velocity).
static void coarse_inverse(Mg &mg, hipStream_t s) {
  MgLevel &L = mg.lv.back();
  const int64_t nodes = L.nodes, m = mg.comps * nodes;
  FSI_REQUIRE(m <= 6000, FSI_E_ARG, "coarsest multigrid level too large: n must be 2^k * m with m <= 6");
  std::vector<int> rp(L.A.nrows + 1), cl(L.A.nnz);
  std::vector<double> v(L.A.nnz * L.A.width);
  FSI_HIP(hipMemcpyAsync(rp.data(), L.A.rowptr.p, rp.size() * 4, hipMemcpyDeviceToHost, s));
  FSI_HIP(hipMemcpyAsync(cl.data(), L.A.col.p, cl.size() * 4, hipMemcpyDeviceToHost, s));
  FSI_HIP(hipMemcpyAsync(v.data(), L.A.val.p, v.size() * 8, hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  std::vector<double> A(m * m, 0.0), X(m * m, 0.0);
  for (int64_t r = 0; r < nodes; ++r)
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      int64_t cc = cl[k];
      if (mg.comps == 2) {
        A[r * m + cc] = v[4 * k];
        A[r * m + nodes + cc] = v[4 * k + 1];
        A[(nodes + r) * m + cc] = v[4 * k + 2];
        A[(nodes + r) * m + nodes + cc] = v[4 * k + 3];
      } else {
        A[r * m + cc] = v[k];
      }
    }
  for (int64_t i = 0; i < m; ++i) X[i * m + i] = 1.0;
  for (int64_t col = 0; col < m; ++col) {
    int64_t piv = col;
    for (int64_t r = col + 1; r < m; ++r)
      if (std::fabs(A[r * m + col]) > std::fabs(A[piv * m + col])) piv = r;
    FSI_REQUIRE(A[piv * m + col] != 0.0, FSI_E_ARG, "singular coarse operator");
    if (piv != col)
      for (int64_t k = 0; k < m; ++k) {
        std::swap(A[piv * m + k], A[col * m + k]);
        std::swap(X[piv * m + k], X[col * m + k]);
      }
    double inv = 1.0 / A[col * m + col];
    for (int64_t k = 0; k < m; ++k) { A[col * m + k] *= inv; X[col * m + k] *= inv; }
    for (int64_t r = 0; r < m; ++r) {
      if (r == col) continue;
      double f = A[r * m + col];
      if (f == 0.0) continue;
      for (int64_t k = 0; k < m; ++k) {
        A[r * m + k] -= f * A[col * m + k];
        X[r * m + k] -= f * X[col * m + k];
      }
    }
  }
  mg.ncoarse = m;
  mg.cinv.alloc(m * m);
  FSI_HIP(hipMemcpyAsync(mg.cinv.p, X.data(), m * m * 8, hipMemcpyHostToDevice, s));
  mg.cinv32.alloc(m * m);
  convert(mg.cinv32.p, mg.cinv.p, m * m, s);
  FSI_HIP(hipStreamSynchronize(s));
}

// The same dense inverse on the device, for symmetric positive definite coarsest operators
// (the Q2 pair's A_f with its Dirichlet identity rows, and L with its pinned identity row):
// Gauss-Jordan elimination without pivoting, one column per step (the pivot row scaled by one
// workgroup, the column's factors copied, then every other row of A and X updated in parallel).
__global__ void k_dense_from_csr(int64_t nodes, int comps, const int *rp, const int *col, const double *v, int64_t m,
                                 double *A) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nodes) return;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int64_t cc = col[k];
    if (comps == 2) {
      A[r * m + cc] = v[4 * (int64_t)k];
      A[r * m + nodes + cc] = v[4 * (int64_t)k + 1];
      A[(nodes + r) * m + cc] = v[4 * (int64_t)k + 2];
      A[(nodes + r) * m + nodes + cc] = v[4 * (int64_t)k + 3];
    } else {
      A[r * m + cc] = v[k];
    }
  }
}

__global__ void k_gj_identity(int64_t m, double *X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) X[i * m + i] = 1.0;
}

// one workgroup: row col of A (from col on: the entries before are zero) and of X divided by the
// pivot, which every thread reads before any is written
__global__ void __launch_bounds__(1024) k_gj_pivot(int64_t m, int64_t col, double *A, double *X) {
  const double inv = 1.0 / A[col * m + col];
  __syncthreads();
  for (int64_t k = col + threadIdx.x; k < m; k += blockDim.x) A[col * m + k] *= inv;
  for (int64_t k = threadIdx.x; k < m; k += blockDim.x) X[col * m + k] *= inv;
}

__global__ void k_gj_factors(int64_t m, int64_t col, const double *A, double *f) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) f[r] = r == col ? 0.0 : A[r * m + col];
}

// row r = blockIdx.y, entry k: A[r][k] -= f[r] A[col][k] (k >= col), X[r][k] -= f[r] X[col][k]
__global__ void k_gj_eliminate(int64_t m, int64_t col, double *A, double *X, const double *f) {
  const int64_t r = blockIdx.y, k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double fr = f[r];
  if (k >= m || fr == 0.0) return;
  if (k >= col) A[r * m + k] -= fr * A[col * m + k];
  X[r * m + k] -= fr * X[col * m + k];
}

static void coarse_inverse_spd_device(Mg &mg, hipStream_t s) {
  MgLevel &L = mg.lv.back();
  const int64_t nodes = L.nodes, m = mg.comps * nodes;
  FSI_REQUIRE(m <= 8192, FSI_E_ARG, "coarsest multigrid level too large for the dense inverse");
  DevBuf<double> A(m * m), f(m);
  mg.cinv.alloc(m * m);
  fill(A.p, m * m, 0.0, s);
  fill(mg.cinv.p, m * m, 0.0, s);
  hipLaunchKernelGGL(k_dense_from_csr, dim3(grid_for(nodes, 256)), dim3(256), 0, s, nodes, mg.comps, L.A.rowptr.p,
                     L.A.col.p, L.A.val.p, m, A.p);
  hipLaunchKernelGGL(k_gj_identity, dim3(grid_for(m, 256)), dim3(256), 0, s, m, mg.cinv.p);
  const dim3 eg((unsigned)((m + 255) / 256), (unsigned)m);
  for (int64_t col = 0; col < m; ++col) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, m, col, A.p, mg.cinv.p);
    hipLaunchKernelGGL(k_gj_factors, dim3(grid_for(m, 256)), dim3(256), 0, s, m, col, A.p, f.p);
    hipLaunchKernelGGL(k_gj_eliminate, eg, dim3(256), 0, s, m, col, A.p, mg.cinv.p, f.p);
  }
  FSI_CHECK_LAUNCH();
  mg.ncoarse = m;
  mg.cinv32.alloc(m * m);
  convert(mg.cinv32.p, mg.cinv.p, m * m, s);
  FSI_HIP(hipStreamSynchronize(s));
}

size_t Mg::bytes() const {
  size_t b = cinv.bytes() + cinv32.bytes() + rtab64.bytes() + rtab32.bytes();
  for (auto &L : lv) {
    b += L.A.bytes() + L.P.bytes() + L.R.bytes() + L.dinv.bytes() + L.dinv32.bytes() + L.stab64.bytes() +
         L.stab32.bytes() + L.p1tab64.bytes() + L.p1tab32.bytes() + L.q2tab64.bytes() + L.q2tab32.bytes();
    for (int i = 0; i < 5; ++i) b += L.w64[i].bytes() + L.w32[i].bytes();
  }
  return b;
}

void build_multigrid(Ctx &c) {
  hipStream_t s = c.stream;
  DevBuf<int> tmp;
  const std::vector<int> ns = mg_level_cells(c.n);
  // velocity: A_f per level (re-discretised = Galerkin for nested P2 spaces)
  c.mgu.comps = 2;
  c.mgp.comps = 1;
  // Chebyshev degrees (steps before and after the coarse correction), from sweeps on the
  // 256^2 / 512^2 / 1024^2 workloads: velocity 3, pressure 2 (pressure degree 3 needed
  // as many or more inner steps: 1024^2 FP64 234 -> 207 inner steps, -13% step time)
  c.mgu.degree = c.mgu.degree32 = 3;
  c.mgp.degree = c.mgp.degree32 = 2;
  // velocity levels: all of them, or from 512^2 on down to the first coarse level of 16^2 or
  // less, whose dense inverse is then formed on the device
  const size_t nu = mg_velocity_levels(ns);
  c.mgu.lv.resize(nu);
  c.mgp.lv.resize(ns.size());
  for (size_t l = 0; l < ns.size(); ++l) {
    int m = ns[l];
    std::vector<double> hE;
    element_tables(m, c.nu, hE);
    DevBuf<double> dE(hE.size());
    FSI_HIP(hipMemcpyAsync(dE.p, hE.data(), hE.size() * 8, hipMemcpyHostToDevice, s));
    // below the velocity coarsest only the pressure level is built (U is then a throw-away
    // level of which only the sizes are set)
    const bool vel = l < nu;
    MgLevel Udummy;
    MgLevel &U = vel ? c.mgu.lv[l] : Udummy;
    MgLevel &P = c.mgp.lv[l];
    U.n = P.n = m;
    U.nodes = (int64_t)(2 * m + 1) * (2 * m + 1);
    P.nodes = (int64_t)(m + 1) * (m + 1);
    if (vel) assemble_p2p2(U.A, nullptr, m, dE.p, c.rho / c.dt, tmp, s);
    assemble_p1p1(P.A, m, dE.p, EM_LP, 1, tmp, s);
    FSI_HIP(hipStreamSynchronize(s));
    P.dinv.alloc(P.nodes);
    if (vel) {
      U.dinv.alloc(4 * U.nodes);
      hipLaunchKernelGGL(k_block_diag_inv, dim3(grid_for(U.nodes, 256)), dim3(256), 0, s, U.nodes, 4,
                         U.A.rowptr.p, U.A.col.p, U.A.val.p, U.dinv.p);
    }
    hipLaunchKernelGGL(k_block_diag_inv, dim3(grid_for(P.nodes, 256)), dim3(256), 0, s, P.nodes, 1,
                       P.A.rowptr.p, P.A.col.p, P.A.val.p, P.dinv.p);
    FSI_CHECK_LAUNCH();
    if (vel) U.lmax = 1.1 * power_lmax(U, 2, s);
    if (vel) {
      StencilTable<double> t64;
      StencilTable<float> t32;
      stencil_tables(m, c.nu, c.rho / c.dt, t64, t32);
      U.stab64.alloc(sizeof(t64));
      U.stab32.alloc(sizeof(t32));
      FSI_HIP(hipMemcpyAsync(U.stab64.p, &t64, sizeof(t64), hipMemcpyHostToDevice, s));
      FSI_HIP(hipMemcpyAsync(U.stab32.p, &t32, sizeof(t32), hipMemcpyHostToDevice, s));
      FSI_HIP(hipStreamSynchronize(s));
    }
    if (m >= 2) {
      P1Table<double> t64;
      P1Table<float> t32;
      p1_tables(m, EM_LP, 1, t64, t32);
      upload_bytes(P.p1tab64, &t64, sizeof(t64), s);
      upload_bytes(P.p1tab32, &t32, sizeof(t32), s);
    }
    P.lmax = 1.1 * power_lmax(P, 1, s);
    if (l + 1 < ns.size()) {
      int64_t nc2 = (int64_t)(m + 1) * (m + 1);          // coarse P2 nodes = (2 (m/2) + 1)^2
      int64_t nc1 = (int64_t)(m / 2 + 1) * (m / 2 + 1);
      unsigned gf2 = grid_for(U.nodes, 256), gc2 = grid_for(nc2, 256);
      if (l + 1 < nu) build_rows(U.P, U.nodes, nc2, 1, s, tmp,
                 [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
                   hipLaunchKernelGGL(k_p2_prolong, dim3(gf2), dim3(256), 0, s, m, pass, cnt, rp, col, v);
                 });
      if (l + 1 < nu) build_rows(U.R, nc2, U.nodes, 1, s, tmp,
                 [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
                   hipLaunchKernelGGL(k_p2_restrict, dim3(gc2), dim3(256), 0, s, m, pass, cnt, rp, col, v);
                 });
      unsigned gf1 = grid_for(P.nodes, 256), gc1 = grid_for(nc1, 256);
      build_rows(P.P, P.nodes, nc1, 1, s, tmp,
                 [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
                   hipLaunchKernelGGL(k_p1_prolong, dim3(gf1), dim3(256), 0, s, m, pass, cnt, rp, col, v);
                 });
      build_rows(P.R, nc1, P.nodes, 1, s, tmp,
                 [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
                   hipLaunchKernelGGL(k_p1_restrict, dim3(gc1), dim3(256), 0, s, m, pass, cnt, rp, col, v);
                 });
    }
    for (int i = 0; i < 5; ++i) {
      if (vel) U.w64[i].alloc(2 * U.nodes);
      P.w64[i].alloc(P.nodes);
    }
  }
  {
    P2RestrTable<double> t64;
    P2RestrTable<float> t32;
    p2_restrict_tables(t64, t32);
    upload_bytes(c.mgu.rtab64, &t64, sizeof(t64), s);
    upload_bytes(c.mgu.rtab32, &t32, sizeof(t32), s);
  }
  if (nu < ns.size()) coarse_inverse_spd_device(c.mgu, s);
  else coarse_inverse(c.mgu, s);
  coarse_inverse(c.mgp, s);
  (void)tail_lds_limit();   // the LDS grant of the coarse-tail launches, outside any graph capture
  FSI_HIP(hipStreamSynchronize(s));
}

// ================================================================ the paper's element pair
// Q2 velocity / discontinuous P1 pressure on the n x n squares (Sec. 4, the discrete spaces).
// The Q2 nodes are the P2 lattice: node (I, J) at (I h/2, J h/2); cell (i, j) holds the nodes
// (2i + a, 2j + b), local index a + 3 b, with the tensor products of the quadratic Lagrange
// polynomials at 0, 1/2, 1; the pressure unknowns of cell k = j n + i are 3k + {0, 1, 2},
// the coefficients of 1, (x - x_c)/h, (y - y_c)/h.  Element integrals by the 3-point Gauss
// rule in each direction, exact for these integrands (degree <= 4 in each variable).
// Element table: M (9 x 9), K[alpha][beta] (4 x 9 x 9, nu eps(phi_j e_beta) : eps(phi_i
// e_alpha) at [alpha][beta][i][j]), B[alpha][k] (2 x 3 x 9, int d_alpha phi_i psi_k), M_p
// diagonal (3: the basis is orthogonal on a square).
void q2_element_table(int n, double nu, std::vector<double> &out) {
  const double h = 1.0 / n;
  out.assign(QE_SIZE, 0.0);
  const double g[3] = {0.5 - std::sqrt(15.0) / 10.0, 0.5, 0.5 + std::sqrt(15.0) / 10.0};
  const double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  auto lag = [](double t, double *v, double *d) {
    v[0] = 2.0 * (t - 0.5) * (t - 1.0);
    v[1] = 4.0 * t * (1.0 - t);
    v[2] = 2.0 * t * (t - 0.5);
    d[0] = 4.0 * t - 3.0;
    d[1] = 4.0 - 8.0 * t;
    d[2] = 4.0 * t - 1.0;
  };
  for (int q = 0; q < 3; ++q)
    for (int p = 0; p < 3; ++p) {
      double vx[3], dx[3], vy[3], dy[3];
      lag(g[p], vx, dx);
      lag(g[q], vy, dy);
      const double wt = w[p] * w[q] * h * h;
      double phi[9], gx[9], gy[9];
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          phi[a + 3 * b] = vx[a] * vy[b];
          gx[a + 3 * b] = dx[a] * vy[b] / h;
          gy[a + 3 * b] = vx[a] * dy[b] / h;
        }
      const double psi[3] = {1.0, g[p] - 0.5, g[q] - 0.5};
      for (int i = 0; i < 9; ++i) {
        const double gi[2] = {gx[i], gy[i]};
        for (int j = 0; j < 9; ++j) {
          const double gj[2] = {gx[j], gy[j]};
          out[QE_M + 9 * i + j] += wt * phi[i] * phi[j];
          // eps(phi_j e_b) : eps(phi_i e_a) = (delta_ab grad phi_j . grad phi_i + d_a phi_j d_b phi_i) / 2
          const double dot = gi[0] * gj[0] + gi[1] * gj[1];
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be)
              out[QE_K + ((al * 2 + be) * 9 + i) * 9 + j] +=
                  wt * 0.5 * nu * ((al == be ? dot : 0.0) + gj[al] * gi[be]);
        }
        for (int k = 0; k < 3; ++k) {
          out[QE_B + (0 * 3 + k) * 9 + i] += wt * gx[i] * psi[k];
          out[QE_B + (1 * 3 + k) * 9 + i] += wt * gy[i] * psi[k];
        }
      }
      for (int k = 0; k < 3; ++k) out[QE_MP + k] += wt * psi[k] * psi[k];
    }
}

// cells [c0, c1] (one direction) whose closure holds lattice line I
__device__ __forceinline__ void q2_cells_of(int I, int n, int &c0, int &c1) {
  c0 = max(0, (I - 1) >> 1);
  c1 = min(n - 1, I >> 1);
}

// Row of A_f (and M_f) at Q2 node (I, J): the nodes of the 1, 2 or 4 cells around it, in
// ascending index; the cells' contributions summed j major, i minor.
__global__ void k_asm_q2q2(int n, int pass, const double *__restrict__ E, double rdt, int *cnt, const int *rowptr,
                           int *col, double *A, double *M) {
  const int64_t L = 2 * n + 1;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  const int I = (int)(row % L), J = (int)(row / L);
  int i0, i1, j0, j1;
  q2_cells_of(I, n, i0, i1);
  q2_cells_of(J, n, j0, j1);
  if (!pass) {
    cnt[row] = (2 * (i1 - i0) + 3) * (2 * (j1 - j0) + 3);
    return;
  }
  const bool rb = p2_boundary(I, J, n);
  int k = rowptr[row];
  for (int J2 = 2 * j0; J2 <= 2 * j1 + 2; ++J2)
    for (int I2 = 2 * i0; I2 <= 2 * i1 + 2; ++I2) {
      double m = 0.0, kk[4] = {0.0, 0.0, 0.0, 0.0};
      for (int cj = j0; cj <= j1; ++cj) {
        const int b = J - 2 * cj, b2 = J2 - 2 * cj;
        if (b2 < 0 || b2 > 2) continue;
        for (int ci = i0; ci <= i1; ++ci) {
          const int a = I - 2 * ci, a2 = I2 - 2 * ci;
          if (a2 < 0 || a2 > 2) continue;
          const int li = a + 3 * b, lj = a2 + 3 * b2;
          m += E[QE_M + 9 * li + lj];
          for (int q = 0; q < 4; ++q) kk[q] += E[QE_K + (q * 9 + li) * 9 + lj];
        }
      }
      col[k] = (int)(J2 * L + I2);
      double *v = A + 4 * (int64_t)k;
      if (rb || p2_boundary(I2, J2, n)) {
        const double d = (I2 == I && J2 == J) ? 1.0 : 0.0;
        v[0] = d; v[1] = 0.0; v[2] = 0.0; v[3] = d;
      } else {
        v[0] = rdt * m + kk[0]; v[1] = kk[1]; v[2] = kk[2]; v[3] = rdt * m + kk[3];
      }
      if (M) M[k] = m;
      ++k;
    }
}

// Row of B at pressure unknown 3k + q: the 9 nodes of cell k (row 0 and boundary columns zero)
__global__ void k_asm_qb(int n, int pass, const double *__restrict__ E, int *cnt, const int *rowptr, int *col,
                         double *V) {
  const int64_t np = 3 * (int64_t)n * n;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= np) return;
  if (!pass) {
    cnt[row] = 9;
    return;
  }
  const int64_t cell = row / 3, L = 2 * n + 1;
  const int q = (int)(row % 3), i = (int)(cell % n), j = (int)(cell / n);
  int k = rowptr[row];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a, ++k) {
      const int I = 2 * i + a, J = 2 * j + b;
      const bool zero = row == 0 || p2_boundary(I, J, n);
      col[k] = (int)(J * L + I);
      V[2 * (int64_t)k] = zero ? 0.0 : E[QE_B + (0 * 3 + q) * 9 + a + 3 * b];
      V[2 * (int64_t)k + 1] = zero ? 0.0 : E[QE_B + (1 * 3 + q) * 9 + a + 3 * b];
    }
}

// Row of B^T at Q2 node (I, J): the pressure unknowns of the cells around it (boundary rows
// and column 0 zero)
__global__ void k_asm_qbt(int n, int pass, const double *__restrict__ E, int *cnt, const int *rowptr, int *col,
                          double *V) {
  const int64_t L = 2 * n + 1;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  const int I = (int)(row % L), J = (int)(row / L);
  int i0, i1, j0, j1;
  q2_cells_of(I, n, i0, i1);
  q2_cells_of(J, n, j0, j1);
  if (!pass) {
    cnt[row] = 3 * (i1 - i0 + 1) * (j1 - j0 + 1);
    return;
  }
  const bool rb = p2_boundary(I, J, n);
  int k = rowptr[row];
  for (int cj = j0; cj <= j1; ++cj)
    for (int ci = i0; ci <= i1; ++ci) {
      const int64_t cell = (int64_t)cj * n + ci;
      const int loc = (I - 2 * ci) + 3 * (J - 2 * cj);
      for (int q = 0; q < 3; ++q, ++k) {
        const int64_t pc = 3 * cell + q;
        const bool zero = rb || pc == 0;
        col[k] = (int)pc;
        V[2 * (int64_t)k] = zero ? 0.0 : E[QE_B + (0 * 3 + q) * 9 + loc];
        V[2 * (int64_t)k + 1] = zero ? 0.0 : E[QE_B + (1 * 3 + q) * 9 + loc];
      }
    }
}

// M_p of the discontinuous pressure: diagonal (one entry per row)
__global__ void k_asm_qmp(int n, int pass, const double *__restrict__ E, int *cnt, const int *rowptr, int *col,
                          double *V) {
  const int64_t np = 3 * (int64_t)n * n;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= np) return;
  if (!pass) {
    cnt[row] = 1;
    return;
  }
  const int k = rowptr[row];
  col[k] = (int)row;
  V[k] = E[QE_MP + row % 3];
}

// row sums (the lumped mass D of M_f)
__global__ void k_row_sum(int64_t nrows, const int *rowptr, const double *v, double *d) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  double s = 0.0;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s += v[k];
  d[r] = s;
}

// Row r of the pressure Laplacian of the discontinuous pair, L = B D^{-1} B^T (D the row sums
// of M_f, B with its Dirichlet columns and pinned row): the unknowns of the cells around r's cell
// (3 x 3 clamped at the boundary), in ascending order; sum over the 9 nodes v of r's cell of
// B_rv . B_sv / D_v.  Row 0 (the pinned unknown) is the identity row.
__global__ void k_q_lp(int n, int pass, const int *__restrict__ brp, const int *__restrict__ bcol,
                       const double *__restrict__ bval, const int *__restrict__ trp, const int *__restrict__ tcol,
                       const double *__restrict__ tval, const double *__restrict__ d, int *cnt, const int *rowptr,
                       int *col, double *V) {
  const int64_t np = 3 * (int64_t)n * n;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= np) return;
  const int64_t cell = r / 3;
  const int ci = (int)(cell % n), cj = (int)(cell / n);
  const int i0 = max(ci - 1, 0), i1 = min(ci + 1, n - 1), j0 = max(cj - 1, 0), j1 = min(cj + 1, n - 1);
  const int wi = i1 - i0 + 1;
  if (!pass) {
    cnt[r] = 3 * wi * (j1 - j0 + 1);
    return;
  }
  const int k0 = rowptr[r];
  for (int j = j0, k = k0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i)
      for (int q = 0; q < 3; ++q, ++k) {
        col[k] = (int)(3 * ((int64_t)j * n + i) + q);
        V[k] = 0.0;
      }
  for (int e = brp[r]; e < brp[r + 1]; ++e) {
    const int v = bcol[e];
    const double bx = bval[2 * (int64_t)e], by = bval[2 * (int64_t)e + 1], dv = d[v];
    if (bx == 0.0 && by == 0.0) continue;
    for (int f = trp[v]; f < trp[v + 1]; ++f) {
      const int sc = tcol[f];
      const int64_t sk = sc / 3;
      const int si = (int)(sk % n), sj = (int)(sk / n);
      V[k0 + 3 * ((sj - j0) * wi + (si - i0)) + sc % 3] += (bx * tval[2 * (int64_t)f] + by * tval[2 * (int64_t)f + 1]) / dv;
    }
  }
  if (r == 0) V[k0] = 1.0;   // the row's first column is unknown 0: B's row 0 left it zero
}

// Prolongation of the discontinuous P1 pressure from an nf / 2 grid into the nf grid: the coarse
// cell's linear function on each of its four children (fine constant = the coarse function at
// the child's centre, x_c +- h_c / 4; fine slopes = half the coarse ones); the pinned unknown 0
// excluded on both grids.
__device__ int pd_prolong_row(int64_t r, int nf, int *cidx, double *w) {
  const int nc = nf / 2;
  const int64_t cell = r / 3;
  const int q = (int)(r % 3), i = (int)(cell % nf), j = (int)(cell / nf);
  const int64_t cc = 3 * ((int64_t)(j >> 1) * nc + (i >> 1));
  const double sx = (i & 1) ? 0.25 : -0.25, sy = (j & 1) ? 0.25 : -0.25;
  int m = 0;
  auto put = [&](int64_t c, double v) {
    if (c == 0) return;
    cidx[m] = (int)c;
    w[m] = v;
    ++m;
  };
  if (q == 0) {
    put(cc, 1.0);
    put(cc + 1, sx);
    put(cc + 2, sy);
  } else {
    put(cc + q, 0.5);
  }
  return m;
}

__global__ void k_pd_prolong(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  const int64_t np = 3 * (int64_t)nf * nf;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= np) return;
  int ci[3];
  double w[3];
  const int m = r == 0 ? 0 : pd_prolong_row(r, nf, ci, w);
  if (!pass) {
    cnt[r] = m;
    return;
  }
  const int k = rowptr[r];
  for (int t = 0; t < m; ++t) {
    col[k + t] = ci[t];
    V[k + t] = w[t];
  }
}

__global__ void k_pd_restrict(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  const int nc = nf / 2;
  const int64_t npc = 3 * (int64_t)nc * nc;
  const int64_t rc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rc >= npc) return;
  const int64_t cell = rc / 3;
  const int ic = (int)(cell % nc), jc = (int)(cell / nc);
  int k = pass ? rowptr[rc] : 0, c = 0;
  if (rc != 0)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int64_t fcell = (int64_t)(2 * jc + dj) * nf + 2 * ic + di;
        for (int q = 0; q < 3; ++q) {
          const int64_t f = 3 * fcell + q;
          if (f == 0) continue;
          int ci[3];
          double w[3];
          const int m = pd_prolong_row(f, nf, ci, w);
          for (int t = 0; t < m; ++t)
            if (ci[t] == rc) {
              if (pass) {
                col[k] = (int)f;
                V[k] = w[t];
                ++k;
              }
              ++c;
            }
        }
      }
  if (!pass) cnt[rc] = c;
}

static void assemble_q2q2(Csr &A, DevBuf<double> *M, int n, const double *dE, double rdt, DevBuf<int> &tmp,
                          hipStream_t s) {
  const int64_t rows = (int64_t)(2 * n + 1) * (2 * n + 1);
  const unsigned g = grid_for(rows, 256);
  build_rows(A, rows, rows, 4, s, tmp,
             [&](int pass, int *cnt, const int *rp, int *col, double *v, double *m) {
               hipLaunchKernelGGL(k_asm_q2q2, dim3(g), dim3(256), 0, s, n, pass, dE, rdt, cnt, rp, col, v, m);
             },
             M != nullptr, M);
}

static DevBuf<double> upload_q2_table(int n, double nu, hipStream_t s) {
  std::vector<double> hE;
  q2_element_table(n, nu, hE);
  DevBuf<double> dE(hE.size());
  FSI_HIP(hipMemcpyAsync(dE.p, hE.data(), hE.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FSI_HIP(hipStreamSynchronize(s));
  return dE;
}

void build_fluid_q2(Ctx &c) {
  hipStream_t s = c.stream;
  const int n = c.n;
  DevBuf<double> dE = upload_q2_table(n, c.nu, s);
  DevBuf<int> tmp;
  assemble_q2q2(c.Af, &c.Mf, n, dE.p, c.rho / c.dt, tmp, s);
  const int64_t np = 3 * (int64_t)n * n, n2 = (int64_t)(2 * n + 1) * (2 * n + 1);
  const unsigned gp = grid_for(np, 256), g2 = grid_for(n2, 256);
  build_rows(c.B, np, n2, 2, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
    hipLaunchKernelGGL(k_asm_qb, dim3(gp), dim3(256), 0, s, n, pass, dE.p, cnt, rp, col, v);
  });
  build_rows(c.BT, n2, np, 2, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
    hipLaunchKernelGGL(k_asm_qbt, dim3(g2), dim3(256), 0, s, n, pass, dE.p, cnt, rp, col, v);
  });
  build_rows(c.Mp, np, np, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
    hipLaunchKernelGGL(k_asm_qmp, dim3(gp), dim3(256), 0, s, n, pass, dE.p, cnt, rp, col, v);
  });
  c.Mp_dinv.alloc(np);
  hipLaunchKernelGGL(k_diag_inv, dim3(gp), dim3(256), 0, s, np, c.Mp.rowptr.p, c.Mp.col.p, c.Mp.val.p,
                     c.Mp_dinv.p);
  c.bnd.alloc(n2);
  hipLaunchKernelGGL(k_p2_boundary_flags, dim3(g2), dim3(256), 0, s, n, c.bnd.p);
  FSI_CHECK_LAUNCH();
  FSI_HIP(hipStreamSynchronize(s));
}


// Coarse Q2 weights at fine lattice node (I, J) of an nf grid: the coarse cell's biquadratic
// basis at the fine node (local coordinates multiples of 1/4: exact binary fractions), interior
// coarse nodes only, in ascending coarse index.
__device__ int q2_prolong_row(int I, int J, int nf, int *cidx, double *w) {
  const int nc = nf / 2;
  const int64_t Lc = 2 * nc + 1;
  const int ci = min(I / 4, nc - 1), cj = min(J / 4, nc - 1);
  const double xi = (I - 4 * ci) * 0.25, eta = (J - 4 * cj) * 0.25;
  const double lx[3] = {2.0 * (xi - 0.5) * (xi - 1.0), 4.0 * xi * (1.0 - xi), 2.0 * xi * (xi - 0.5)};
  const double ly[3] = {2.0 * (eta - 0.5) * (eta - 1.0), 4.0 * eta * (1.0 - eta), 2.0 * eta * (eta - 0.5)};
  int cnt = 0;
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) {
      const double wt = lx[a] * ly[b];
      if (wt == 0.0) continue;
      const int Ic = 2 * ci + a, Jc = 2 * cj + b;
      if (p2_boundary(Ic, Jc, nc)) continue;
      cidx[cnt] = (int)(Jc * Lc + Ic);
      w[cnt] = wt;
      ++cnt;
    }
  return cnt;
}

__global__ void k_q2_prolong(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  const int64_t L = 2 * nf + 1;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L * L) return;
  const int I = (int)(row % L), J = (int)(row / L);
  int ci[9];
  double w[9];
  const int m = p2_boundary(I, J, nf) ? 0 : q2_prolong_row(I, J, nf, ci, w);
  if (!pass) {
    cnt[row] = m;
    return;
  }
  const int k = rowptr[row];
  for (int q = 0; q < m; ++q) {
    col[k + q] = ci[q];
    V[k + q] = w[q];
  }
}

__global__ void k_q2_restrict(int nf, int pass, int *cnt, const int *rowptr, int *col, double *V) {
  const int nc = nf / 2;
  const int64_t Lc = 2 * nc + 1, L = 2 * nf + 1;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Lc * Lc) return;
  const int Ic = (int)(row % Lc), Jc = (int)(row / Lc);
  int k = pass ? rowptr[row] : 0, c = 0;
  if (!p2_boundary(Ic, Jc, nc)) {
    for (int J = 2 * Jc - 4; J <= 2 * Jc + 4; ++J)
      for (int I = 2 * Ic - 4; I <= 2 * Ic + 4; ++I) {
        if (I < 0 || J < 0 || I > 2 * nf || J > 2 * nf || p2_boundary(I, J, nf)) continue;
        int ci[9];
        double w[9];
        const int m = q2_prolong_row(I, J, nf, ci, w);
        for (int q = 0; q < m; ++q)
          if (ci[q] == row) {
            if (pass) {
              col[k] = (int)((int64_t)J * L + I);
              V[k] = w[q];
              ++k;
            }
            ++c;
          }
      }
  }
  if (!pass) cnt[row] = c;
}

// The hierarchies of the Q2 pair, smoothed on the assembled operators (no matrix-free form):
// velocity, A_f re-discretised on every level (the Galerkin operator of the nested Q2 spaces)
// with the biquadratic prolongation and its transpose; pressure, L = B D^{-1} B^T of each level
// (the Laplacian of the Cahouet-Chabard approximation for a discontinuous pressure) with the
// P1-disc prolongation and its transpose; dense inverses at the coarsest level.
void build_multigrid_q2(Ctx &c) {
  hipStream_t s = c.stream;
  DevBuf<int> tmp;
  std::vector<int> ns;
  for (int m = c.n;; m /= 2) {
    ns.push_back(m);
    // the coarsest level at 16^2 or below (dense inverses of at most 2,178 velocity and 768
    // pressure unknowns, formed on the device): the levels below 32^2 are launch latency, and
    // the exact solve there also cuts the inner steps (256^2 bar: 114 against 151 per step)
    if (m <= 16 || (m & 1)) break;
  }
  c.mgu.comps = 2;
  c.mgu.degree = c.mgu.degree32 = 3;
  c.mgu.stencil = false;
  c.mgu.tail = false;
  c.mgu.lv.resize(ns.size());
  c.mgp.comps = 1;
  c.mgp.degree = c.mgp.degree32 = 2;
  c.mgp.stencil = false;
  c.mgp.tail = false;
  c.mgp.lv.resize(ns.size());
  for (size_t l = 0; l < ns.size(); ++l) {
    const int m = ns[l];
    DevBuf<double> dE = upload_q2_table(m, c.nu, s);
    MgLevel &U = c.mgu.lv[l];
    U.n = m;
    U.nodes = (int64_t)(2 * m + 1) * (2 * m + 1);
    DevBuf<double> Ml;
    assemble_q2q2(U.A, &Ml, m, dE.p, c.rho / c.dt, tmp, s);
    FSI_HIP(hipStreamSynchronize(s));
    {   // the pressure level: L = B D^{-1} B^T from this level's B, B^T and lumped M_f
      MgLevel &P = c.mgp.lv[l];
      P.n = m;
      P.nodes = 3 * (int64_t)m * m;
      const unsigned gp = grid_for(P.nodes, 256), g2 = grid_for(U.nodes, 256);
      Csr Bl, BTl;
      build_rows(Bl, P.nodes, U.nodes, 2, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
        hipLaunchKernelGGL(k_asm_qb, dim3(gp), dim3(256), 0, s, m, pass, dE.p, cnt, rp, col, v);
      });
      build_rows(BTl, U.nodes, P.nodes, 2, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
        hipLaunchKernelGGL(k_asm_qbt, dim3(g2), dim3(256), 0, s, m, pass, dE.p, cnt, rp, col, v);
      });
      DevBuf<double> d(U.nodes);
      hipLaunchKernelGGL(k_row_sum, dim3(g2), dim3(256), 0, s, U.nodes, U.A.rowptr.p, Ml.p, d.p);
      build_rows(P.A, P.nodes, P.nodes, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
        hipLaunchKernelGGL(k_q_lp, dim3(gp), dim3(256), 0, s, m, pass, Bl.rowptr.p, Bl.col.p, Bl.val.p, BTl.rowptr.p,
                           BTl.col.p, BTl.val.p, d.p, cnt, rp, col, v);
      });
      FSI_HIP(hipStreamSynchronize(s));
      P.dinv.alloc(P.nodes);
      hipLaunchKernelGGL(k_block_diag_inv, dim3(gp), dim3(256), 0, s, P.nodes, 1, P.A.rowptr.p, P.A.col.p, P.A.val.p,
                         P.dinv.p);
      FSI_CHECK_LAUNCH();
      P.lmax = 1.1 * power_lmax(P, 1, s);
      if (l + 1 < ns.size()) {
        const int64_t npc = 3 * (int64_t)(m / 2) * (m / 2);
        build_rows(P.P, P.nodes, npc, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
          hipLaunchKernelGGL(k_pd_prolong, dim3(gp), dim3(256), 0, s, m, pass, cnt, rp, col, v);
        });
        build_rows(P.R, npc, P.nodes, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
          hipLaunchKernelGGL(k_pd_restrict, dim3(grid_for(npc, 256)), dim3(256), 0, s, m, pass, cnt, rp, col, v);
        });
      }
      for (int i = 0; i < 5; ++i) P.w64[i].alloc(P.nodes);
      FSI_HIP(hipStreamSynchronize(s));   // the level's B, B^T and D are freed below
    }
    U.dinv.alloc(4 * U.nodes);
    hipLaunchKernelGGL(k_block_diag_inv, dim3(grid_for(U.nodes, 256)), dim3(256), 0, s, U.nodes, 4, U.A.rowptr.p,
                       U.A.col.p, U.A.val.p, U.dinv.p);
    FSI_CHECK_LAUNCH();
    U.lmax = 1.1 * power_lmax(U, 2, s);
    if (m >= 2) {   // the class stencils of the smoothing steps and residuals
      Q2Table<double> t64;
      Q2Table<float> t32;
      q2_tables(m, c.nu, c.rho / c.dt, t64, t32);
      upload_bytes(U.q2tab64, &t64, sizeof(t64), s);
      upload_bytes(U.q2tab32, &t32, sizeof(t32), s);
    }
    if (l + 1 < ns.size()) {
      const int64_t nc2 = (int64_t)(m + 1) * (m + 1);
      const unsigned gf2 = grid_for(U.nodes, 256), gc2 = grid_for(nc2, 256);
      build_rows(U.P, U.nodes, nc2, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
        hipLaunchKernelGGL(k_q2_prolong, dim3(gf2), dim3(256), 0, s, m, pass, cnt, rp, col, v);
      });
      build_rows(U.R, nc2, U.nodes, 1, s, tmp, [&](int pass, int *cnt, const int *rp, int *col, double *v, double *) {
        hipLaunchKernelGGL(k_q2_restrict, dim3(gc2), dim3(256), 0, s, m, pass, cnt, rp, col, v);
      });
    }
    for (int i = 0; i < 5; ++i) U.w64[i].alloc(2 * U.nodes);
  }
  coarse_inverse_spd_device(c.mgu, s);
  coarse_inverse_spd_device(c.mgp, s);
  FSI_HIP(hipStreamSynchronize(s));
}

}  // namespace fsi
