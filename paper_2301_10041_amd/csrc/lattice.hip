// Matrix-free multigrid pieces on the structured grid: P1 pressure operators, the first
// Chebyshev step with class-wise diagonal inverses, and P2 / P1 grid transfers.  Each
// equals the corresponding assembled (CSR) product up to the order of the sums; the CSR
// path stays available and serves as the reference in the tests.
//
// Bytes per node (scalar values of width w per component):
//   P1 Chebyshev step   x, b, d read; d, y written           5 w
//   first step          b read; d, x written                 3 w per component
//   P2 prolongation-add fine y read and written, coarse x    (2 + 1/4) w per component
//   (the P2 restriction runs with the residual in resid_restrict, stencil.hip; the P2
//   restriction weights are built here)
#include <cstring>

#include "kernels.h"
#include "lattice.h"

namespace fsi {

// Every kernel below runs K independent systems (lane = blockIdx.y) over per-lane views (LP).

// ---------------------------------------------------------------- P1 operators
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_p1(int n, const P1Table<T> *__restrict__ tabp, LP<const T> xl,
                                            LP<const T> bl, LP<T> dl, LP<T> yl, T c1, T c2) {
  const T *__restrict__ x = xl.at(blockIdx.y), *__restrict__ b = bl.at(blockIdx.y);
  T *d = dl.at(blockIdx.y), *y = yl.at(blockIdx.y);
  const int L = n + 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)L * L) return;
  const int i = (int)(r % L), j = (int)(r / L);
  const P1Table<T> &tb = *tabp;
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  const int cls = 3 * cj + ci;
  const bool pin = tb.pin != 0;
  const T xc = x[r];
  T s;
  if (pin && r == 0) {
    s = xc;                                    // identity row of the pinned node
  } else {
    const T *c = tb.coef[cls];
    // column 0 is zero when pinned: its value is read as 0
    auto ld = [&](int64_t q) -> T { return (pin && q == 0) ? T(0) : x[q]; };
    s = c[0] * xc;
    if (i > 0) s += c[1] * ld(r - 1);
    if (i < n) s += c[2] * x[r + 1];
    if (j > 0) s += c[3] * ld(r - L);
    if (j < n) s += c[4] * x[r + L];
    if (i > 0 && j > 0) s += c[5] * ld(r - L - 1);
    if (i < n && j < n) s += c[6] * x[r + L + 1];
  }
  if constexpr (MODE == SP_APPLY) {
    y[r] = s;
  } else if constexpr (MODE == SP_RESID) {
    y[r] = b[r] - s;
  } else {
    const T z = tb.dinv[cls] * (b[r] - s);
    const T dn = c1 * d[r] + c2 * z;
    d[r] = dn;
    y[r] = xc + dn;
  }
}

template <typename T, int MODE>
void p1_launch(int n, const P1Table<T> *tab, LP<const T> x, LP<const T> b, LP<T> d, LP<T> y, T c1, T c2,
               hipStream_t s, int K) {
  const int64_t nodes = (int64_t)(n + 1) * (n + 1);
  hipLaunchKernelGGL((k_p1<T, MODE>), dim3(grid_for(nodes, 256), K), dim3(256), 0, s, n, tab, x, b, d, y, c1, c2);
  FSI_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_p1_first(int n, const P1Table<T> *__restrict__ tabp, LP<const T> bl, T scale, LP<T> dl,
                           LP<T> xl) {
  const T *__restrict__ b = bl.at(blockIdx.y);
  T *d = dl.at(blockIdx.y), *x = xl.at(blockIdx.y);
  const int L = n + 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)L * L) return;
  const int i = (int)(r % L), j = (int)(r / L);
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  const T z = scale * (tabp->dinv[3 * cj + ci] * b[r]);
  d[r] = z;
  x[r] = z;
}

template <typename T>
void p1_first(int n, const P1Table<T> *tab, LP<const T> b, T scale, LP<T> d, LP<T> x, hipStream_t s, int K) {
  const int64_t nodes = (int64_t)(n + 1) * (n + 1);
  hipLaunchKernelGGL(k_p1_first<T>, dim3(grid_for(nodes, 256), K), dim3(256), 0, s, n, tab, b, scale, d, x);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- P2 first Chebyshev step
template <typename T>
__global__ void k_p2_first(int n, const StencilTable<T> *__restrict__ tabp, LP<const T> bl, T scale, LP<T> dl,
                           LP<T> xl) {
  const T *__restrict__ b = bl.at(blockIdx.y);
  T *d = dl.at(blockIdx.y), *x = xl.at(blockIdx.y);
  const int L = 2 * n + 1;
  const int64_t N = (int64_t)L * L;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int I = (int)(r % L), J = (int)(r / L);
  const T b0 = b[r], b1 = b[N + r];
  T z0, z1;
  if (I == 0 || J == 0 || I == 2 * n || J == 2 * n) {
    z0 = scale * b0;                           // identity rows (Dirichlet nodes)
    z1 = scale * b1;
  } else {
    const T *di = tabp->dinv[(I & 1) | ((J & 1) << 1)];
    z0 = scale * (di[0] * b0 + di[1] * b1);
    z1 = scale * (di[2] * b0 + di[3] * b1);
  }
  d[r] = z0;
  x[r] = z0;
  d[N + r] = z1;
  x[N + r] = z1;
}

template <typename T>
void p2_first(int n, const StencilTable<T> *tab, LP<const T> b, T scale, LP<T> d, LP<T> x, hipStream_t s,
              int K) {
  const int64_t nodes = (int64_t)(2 * n + 1) * (2 * n + 1);
  hipLaunchKernelGGL(k_p2_first<T>, dim3(grid_for(nodes, 256), K), dim3(256), 0, s, n, tab, b, scale, d, x);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- P2 transfers
__device__ __forceinline__ bool on_p2_boundary(int I, int J, int n) {
  return I == 0 || J == 0 || I == 2 * n || J == 2 * n;
}

// y += P xc: coarse quadratic evaluated at the fine node; Dirichlet nodes (fine rows and
// coarse columns) take no part.  An interior fine node (I, J) lies in coarse cell
// (I >> 2, J >> 2) at the local position (I mod 4, J mod 4): one of 16 classes, each a fixed
// set of at most six coarse nodes and weights (prolong_classes).
struct ProlongClass {
  int cnt;
  int d[6][2];    // coarse lattice offsets from (2 ci, 2 cj)
  double w[6];    // basis values (exact binary fractions)
};
struct ProlongClasses {
  ProlongClass c[16];   // index 4 (J mod 4) + (I mod 4)
};
__host__ __device__ constexpr ProlongClasses prolong_classes() {
  ProlongClasses t{};
  const int vx[2][3] = {{0, 2, 2}, {0, 2, 0}};
  const int vy[2][3] = {{0, 0, 2}, {0, 2, 2}};
  for (int B = 0; B < 4; ++B)
    for (int A = 0; A < 4; ++A) {
      ProlongClass &p = t.c[4 * B + A];
      const double xi = 0.25 * A, eta = 0.25 * B;
      const int tr = xi >= eta ? 0 : 1;
      const double l0 = tr == 0 ? 1.0 - xi : 1.0 - eta, l1 = tr == 0 ? xi - eta : xi,
                   l2 = tr == 0 ? eta : eta - xi;
      const double phi[6] = {l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                             4 * l0 * l1,       4 * l1 * l2,       4 * l2 * l0};
      p.cnt = 0;
      for (int b = 0; b < 6; ++b) {
        if (phi[b] == 0.0) continue;
        int dI = 0, dJ = 0;
        if (b < 3) {
          dI = vx[tr][b];
          dJ = vy[tr][b];
        } else {
          const int e = b - 3, f = (e + 1) % 3;
          dI = (vx[tr][e] + vx[tr][f]) / 2;
          dJ = (vy[tr][e] + vy[tr][f]) / 2;
        }
        p.d[p.cnt][0] = dI;
        p.d[p.cnt][1] = dJ;
        p.w[p.cnt] = phi[b];
        ++p.cnt;
      }
    }
  return t;
}

// One fine row segment per block, one node per thread (lanes on consecutive nodes: coalesced
// reads and writes of y).  The row's J mod 4 = B is uniform over the block; the node's
// I mod 4 varies with the lane, so each of the six (offset, weight) entries is selected from
// the four compile-time classes of the row (unused entries: weight 0 at the cell's first
// node).  Coarse Dirichlet nodes read as 0.  Sums in the order of prolong_classes.
template <typename T, int B>
__device__ __forceinline__ void prolong_row(int I, int J, int nc, int Lc, int64_t Nc, const T *__restrict__ xc, T &s0,
                                            T &s1) {
  constexpr ProlongClasses pcs = prolong_classes();
  const int A = I & 3, ci = I >> 2, cj = J >> 2;
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    auto pick_i = [&](int a) { return q < pcs.c[4 * B + a].cnt ? pcs.c[4 * B + a].d[q][0] : 0; };
    auto pick_j = [&](int a) { return q < pcs.c[4 * B + a].cnt ? pcs.c[4 * B + a].d[q][1] : 0; };
    auto pick_w = [&](int a) { return q < pcs.c[4 * B + a].cnt ? pcs.c[4 * B + a].w[q] : 0.0; };
    const int dI = A == 0 ? pick_i(0) : A == 1 ? pick_i(1) : A == 2 ? pick_i(2) : pick_i(3);
    const int dJ = A == 0 ? pick_j(0) : A == 1 ? pick_j(1) : A == 2 ? pick_j(2) : pick_j(3);
    const T w = (T)(A == 0 ? pick_w(0) : A == 1 ? pick_w(1) : A == 2 ? pick_w(2) : pick_w(3));
    const int Ic = 2 * ci + dI, Jc = 2 * cj + dJ;
    const bool in = Ic > 0 && Jc > 0 && Ic < 2 * nc && Jc < 2 * nc;
    const int64_t k = in ? (int64_t)Jc * Lc + Ic : 0;
    const T v0 = in ? xc[k] : T(0), v1 = in ? xc[Nc + k] : T(0);
    s0 += w * v0;
    s1 += w * v1;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_p2_prolong_add(int nf, LP<const T> xcl, LP<T> yl, int segs) {
  const T *__restrict__ xc = xcl.at(blockIdx.y);
  T *y = yl.at(blockIdx.y);
  const int L = 2 * nf + 1, nc = nf / 2, Lc = 2 * nc + 1;
  const int64_t Nf = (int64_t)L * L, Nc = (int64_t)Lc * Lc;
  const int J = blockIdx.x / segs, seg = blockIdx.x % segs;
  const int I = seg * 256 + (int)threadIdx.x;
  if (I >= L || I == 0 || J == 0 || I == 2 * nf || J == 2 * nf) return;
  T s0, s1;
  switch (J & 3) {
    case 0: prolong_row<T, 0>(I, J, nc, Lc, Nc, xc, s0, s1); break;
    case 1: prolong_row<T, 1>(I, J, nc, Lc, Nc, xc, s0, s1); break;
    case 2: prolong_row<T, 2>(I, J, nc, Lc, Nc, xc, s0, s1); break;
    default: prolong_row<T, 3>(I, J, nc, Lc, Nc, xc, s0, s1); break;
  }
  const int64_t r = (int64_t)J * L + I;
  y[r] += s0;
  y[Nf + r] += s1;
}

template <typename T>
void p2_prolong_add(int nf, LP<const T> xc, LP<T> y, hipStream_t s, int K) {
  const int L = 2 * nf + 1;
  const int segs = (L + 255) / 256;
  hipLaunchKernelGGL(k_p2_prolong_add<T>, dim3((unsigned)(L * segs), K), dim3(256), 0, s, nf, xc, y, segs);
  FSI_CHECK_LAUNCH();
}

// Host: the restriction weights do not depend on the level (nested uniform refinement),
// so they are read off at interior coarse nodes of a 16 x 16 fine grid.
void p2_restrict_tables(P2RestrTable<double> &t64, P2RestrTable<float> &t32) {
  std::memset(&t64, 0, sizeof(t64));
  std::memset(&t32, 0, sizeof(t32));
  const int nf = 16;
  for (int cls = 0; cls < 4; ++cls) {
    const int Ic = 4 + (cls & 1), Jc = 4 + (cls >> 1);
    int cnt = 0;
    for (int dJ = -4; dJ <= 4; ++dJ)
      for (int dI = -4; dI <= 4; ++dI) {
        int ic[6], jc[6];
        double w[6];
        const int m = p2_prolong_weights(2 * Ic + dI, 2 * Jc + dJ, nf, ic, jc, w);
        for (int q = 0; q < m; ++q)
          if (ic[q] == Ic && jc[q] == Jc) {
            FSI_REQUIRE(cnt < kRestrMax, FSI_E_ARG, "restriction table overflow");
            t64.off[cls][cnt][0] = t32.off[cls][cnt][0] = dI;
            t64.off[cls][cnt][1] = t32.off[cls][cnt][1] = dJ;
            t64.w[cls][cnt] = w[q];
            t32.w[cls][cnt] = (float)w[q];
            ++cnt;
          }
      }
    t64.count[cls] = t32.count[cls] = cnt;
    constexpr RestrOffsets ro = restrict_offsets();
    FSI_REQUIRE(cnt == kRestrCount[cls], FSI_E_ARG, "unexpected restriction width");
    for (int k = 0; k < cnt; ++k)
      FSI_REQUIRE(t64.off[cls][k][0] == ro.d[cls][k][0] && t64.off[cls][k][1] == ro.d[cls][k][1], FSI_E_ARG,
                  "restriction offsets differ from the compiled pattern");
  }
  // the compiled prolongation classes against the interpolation they stand for
  constexpr ProlongClasses pcs = prolong_classes();
  for (int c = 0; c < 16; ++c) {
    const int ci = 3, cj = 3, I = 4 * ci + (c & 3), J = 4 * cj + (c >> 2);
    int ic[6], jc[6];
    double w[6];
    const int m = p2_prolong_weights(I, J, nf, ic, jc, w);
    FSI_REQUIRE(m == pcs.c[c].cnt, FSI_E_ARG, "prolongation class width differs from the interpolation");
    for (int q = 0; q < m; ++q)
      FSI_REQUIRE(ic[q] == 2 * ci + pcs.c[c].d[q][0] && jc[q] == 2 * cj + pcs.c[c].d[q][1] && w[q] == pcs.c[c].w[q],
                  FSI_E_ARG, "prolongation class differs from the interpolation");
  }
}

// ---------------------------------------------------------------- P1 transfers
// Linear interpolation on the nested triangulation; the pinned node 0 is excluded on both
// grids (fine row 0 and coarse column 0 are empty).
template <typename T>
__global__ void __launch_bounds__(256) k_p1_prolong_add(int nf, LP<const T> xcl, LP<T> yl) {
  const T *__restrict__ xc = xcl.at(blockIdx.y);
  T *y = yl.at(blockIdx.y);
  const int L = nf + 1, Lc = nf / 2 + 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0 || r >= (int64_t)L * L) return;
  const int i = (int)(r % L), j = (int)(r / L), ci = i >> 1, cj = j >> 1;
  auto cv = [&](int a, int bb) -> T {
    const int64_t k = (int64_t)bb * Lc + a;
    return k == 0 ? T(0) : xc[k];
  };
  T s;
  if (!(i & 1) && !(j & 1)) s = cv(ci, cj);
  else if (!(j & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj);
  else if (!(i & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci, cj + 1);
  else s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj + 1);
  y[r] += s;
}

template <typename T>
void p1_prolong_add(int nf, LP<const T> xc, LP<T> y, hipStream_t s, int K) {
  const int64_t nodes = (int64_t)(nf + 1) * (nf + 1);
  hipLaunchKernelGGL(k_p1_prolong_add<T>, dim3(grid_for(nodes, 256), K), dim3(256), 0, s, nf, xc, y);
  FSI_CHECK_LAUNCH();
}

// Coarse node (ic, jc) collects the fine node on it (weight 1) and the six fine edge
// midpoints around it (weight 1/2): horizontal, vertical and the two along the cell
// diagonals through it.
template <typename T>
__global__ void __launch_bounds__(256) k_p1_restrict(int nf, LP<const T> rl, LP<T> bcl) {
  const T *__restrict__ r = rl.at(blockIdx.y);
  T *bc = bcl.at(blockIdx.y);
  const int L = nf + 1, Lc = nf / 2 + 1;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)Lc * Lc) return;
  if (q == 0) {
    bc[0] = T(0);
    return;
  }
  const int fi = 2 * (int)(q % Lc), fj = 2 * (int)(q / Lc);
  auto fv = [&](int a, int bb) -> T {
    if (a < 0 || bb < 0 || a > nf || bb > nf) return T(0);
    const int64_t f = (int64_t)bb * L + a;
    return f == 0 ? T(0) : r[f];
  };
  const T edges = fv(fi - 1, fj) + fv(fi + 1, fj) + fv(fi, fj - 1) + fv(fi, fj + 1) + fv(fi + 1, fj + 1) +
                  fv(fi - 1, fj - 1);
  bc[q] = fv(fi, fj) + T(0.5) * edges;
}

template <typename T>
void p1_restrict(int nf, LP<const T> r, LP<T> bc, hipStream_t s, int K) {
  const int64_t nodes = (int64_t)(nf / 2 + 1) * (nf / 2 + 1);
  hipLaunchKernelGGL(k_p1_restrict<T>, dim3(grid_for(nodes, 256), K), dim3(256), 0, s, nf, r, bc);
  FSI_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- P1 Chebyshev steps in one launch
// S steps of the Chebyshev recurrence of chebyshev_p1 on a P1 operator in one launch, on a
// tile of kP1T rows x kP1C nodes: from zero the first step is pointwise (x = d = c2[0]
// D^{-1} b), else the first step starts from x with the direction coefficient c1[0] = 0.  The
// right-hand side (and x) are staged with a halo of S - 1 (S from x); step k runs on the tile
// plus a halo of S - 1 - k, reading x from LDS and writing the next x to the other LDS buffer;
// b and the direction of a node stay in the registers of the thread that owns it.  The
// products keep the order of sums of k_p1 (and its boundary classes, pinned row and column).
// OUT: the result to y (P1_OUT_X), or (P1_OUT_SCHUR) z = a x + b2 w, the pinned entry r[0]
// (rounded through T), and per tile the part of the sum of r z (r64 when given), the output
// stage of the Cahouet-Chabard approximation (x the mass solve, w the Laplacian cycle).
template <typename T, typename TZ, int S, bool ZERO, int OUT>
__global__ void __launch_bounds__(256) k_p1_multi(P1MultiArgs<T, TZ> a, int tiles_x) {
  constexpr int H = ZERO ? S - 1 : S;
  constexpr int RH = kP1T + 2 * H, RW = kP1C + 2 * H, NE = RH * RW, IT = (NE + 255) / 256;
  __shared__ T XA[NE], XB[NE];
  const int lane = blockIdx.y, tid = threadIdx.x;
  const T *b = a.b + lane * a.lb;
  const int n = a.n, L = n + 1;
  const int i0 = (blockIdx.x % tiles_x) * kP1C, j0 = (blockIdx.x / tiles_x) * kP1T;
  const P1Table<T> &tb = *a.tab;
  const bool pin = tb.pin != 0;
  T bq[IT], dq[IT];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + 256 * q, i = i0 - H + e % RW, j = j0 - H + e / RW;
    const bool ok = e < NE && i >= 0 && j >= 0 && i <= n && j <= n;
    bq[q] = ok ? b[(int64_t)j * L + i] : T(0);
    dq[q] = T(0);
    if constexpr (!ZERO) {
      if (e < NE) XA[e] = ok ? a.x[lane * a.lb + (int64_t)j * L + i] : T(0);
    }
  }
  // a node takes part in step k when it lies within S - 1 - k of the tile
  auto ring = [&](int i, int j) {
    const int di = i < i0 ? i0 - i : (i >= i0 + kP1C ? i - (i0 + kP1C - 1) : 0);
    const int dj = j < j0 ? j0 - j : (j >= j0 + kP1T ? j - (j0 + kP1T - 1) : 0);
    return di > dj ? di : dj;
  };
  if constexpr (ZERO) {
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + 256 * q, i = i0 - H + e % RW, j = j0 - H + e / RW;
      if (e < NE) {
        T z = T(0);
        if (i >= 0 && j >= 0 && i <= n && j <= n) {
          const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
          z = a.c2[0] * (tb.dinv[3 * cj + ci] * bq[q]);
        }
        dq[q] = z;
        XA[e] = z;
      }
    }
  }
  __syncthreads();
  T res[IT];   // results of the last step (tile nodes)
  constexpr int K0 = ZERO ? 1 : 0;
#pragma unroll
  for (int k = K0; k < S; ++k) {
    const T *X = ((k - K0) & 1) ? XB : XA;
    T *Xn = ((k - K0) & 1) ? XA : XB;
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + 256 * q, i = i0 - H + e % RW, j = j0 - H + e / RW;
      if (e >= NE || i < 0 || j < 0 || i > n || j > n || ring(i, j) > S - 1 - k) continue;
      const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
      const int cls = 3 * cj + ci;
      const int64_t r = (int64_t)j * L + i;
      const T xc = X[e];
      T sum;
      if (pin && r == 0) {
        sum = xc;   // identity row of the pinned node
      } else {
        const T *c = tb.coef[cls];
        // column 0 is zero when pinned: node (0, 0) is read as 0
        auto ld = [&](int o, int64_t g) -> T { return (pin && g == 0) ? T(0) : X[o]; };
        sum = c[0] * xc;
        if (i > 0) sum += c[1] * ld(e - 1, r - 1);
        if (i < n) sum += c[2] * X[e + 1];
        if (j > 0) sum += c[3] * ld(e - RW, r - L);
        if (j < n) sum += c[4] * X[e + RW];
        if (i > 0 && j > 0) sum += c[5] * ld(e - RW - 1, r - L - 1);
        if (i < n && j < n) sum += c[6] * X[e + RW + 1];
      }
      const T z = tb.dinv[cls] * (bq[q] - sum);
      const T dn = a.c1[k] * dq[q] + a.c2[k] * z;
      dq[q] = dn;
      if (k < S - 1) Xn[e] = xc + dn;
      else res[q] = xc + dn;
    }
    if (k < S - 1) __syncthreads();
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int e = tid + 256 * q, i = i0 - H + e % RW, j = j0 - H + e / RW;
    if (e >= NE || i < 0 || j < 0 || i > n || j > n || ring(i, j) > 0) continue;
    const int64_t r = (int64_t)j * L + i;
    if constexpr (OUT == P1_OUT_X) {
      a.y[lane * a.lb + r] = res[q];
    } else {
      const TZ *rr = a.r + lane * a.lz;
      const TZ v = (TZ)(r == 0 ? (T)rr[0] : a.a * res[q] + a.b2 * a.w[lane * a.lb + r]);
      a.z[lane * a.lz + r] = v;
      acc += (a.r64 ? a.r64[lane * a.lz + r] : (double)rr[r]) * (double)v;
    }
  }
  if constexpr (OUT == P1_OUT_SCHUR) {
    if (a.part) {
      const double t = block_sum(acc);
      if (tid == 0) a.part[lane * a.lp + blockIdx.x] = t;
    }
  }
}

int p1_multi_tiles(int n) {
  const int L = n + 1;
  return ((L + kP1C - 1) / kP1C) * ((L + kP1T - 1) / kP1T);
}

template <typename T, typename TZ, int S, bool ZERO, int OUT>
void p1_multi(const P1MultiArgs<T, TZ> &a, hipStream_t s, int K) {
  const int L = a.n + 1, tx = (L + kP1C - 1) / kP1C;
  hipLaunchKernelGGL((k_p1_multi<T, TZ, S, ZERO, OUT>), dim3((unsigned)p1_multi_tiles(a.n), (unsigned)K), dim3(256),
                     0, s, a, tx);
  FSI_CHECK_LAUNCH();
}

#define FSI_LATTICE_INST(T)                                                                                 \
  template void p1_launch<T, SP_APPLY>(int, const P1Table<T> *, LP<const T>, LP<const T>, LP<T>, LP<T>, T, T, \
                                       hipStream_t, int);                                                   \
  template void p1_launch<T, SP_RESID>(int, const P1Table<T> *, LP<const T>, LP<const T>, LP<T>, LP<T>, T, T, \
                                       hipStream_t, int);                                                   \
  template void p1_launch<T, SP_CHEB>(int, const P1Table<T> *, LP<const T>, LP<const T>, LP<T>, LP<T>, T, T,  \
                                      hipStream_t, int);                                                    \
  template void p1_first<T>(int, const P1Table<T> *, LP<const T>, T, LP<T>, LP<T>, hipStream_t, int);        \
  template void p2_first<T>(int, const StencilTable<T> *, LP<const T>, T, LP<T>, LP<T>, hipStream_t, int);   \
  template void p2_prolong_add<T>(int, LP<const T>, LP<T>, hipStream_t, int);                               \
  template void p1_prolong_add<T>(int, LP<const T>, LP<T>, hipStream_t, int);                               \
  template void p1_restrict<T>(int, LP<const T>, LP<T>, hipStream_t, int);                                  \
  template void p1_multi<T, T, 2, true, P1_OUT_X>(const P1MultiArgs<T, T> &, hipStream_t, int);              \
  template void p1_multi<T, T, 2, false, P1_OUT_X>(const P1MultiArgs<T, T> &, hipStream_t, int);             \
  template void p1_multi<T, T, 3, true, P1_OUT_X>(const P1MultiArgs<T, T> &, hipStream_t, int);              \
  template void p1_multi<T, T, 3, false, P1_OUT_X>(const P1MultiArgs<T, T> &, hipStream_t, int);             \
  template void p1_multi<T, T, 3, true, P1_OUT_SCHUR>(const P1MultiArgs<T, T> &, hipStream_t, int);

FSI_LATTICE_INST(double)
FSI_LATTICE_INST(float)
template void p1_multi<float, double, 3, true, P1_OUT_SCHUR>(const P1MultiArgs<float, double> &, hipStream_t, int);

}  // namespace fsi
