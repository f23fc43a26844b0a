// The coarse end of the velocity V-cycle in one launch per system (Sec. 4 multigrid).  On
// levels of at most 16 x 16 cells every smoothing step, residual and transfer of the
// separate launches costs the latency of a whole kernel while the level holds a few
// thousand nodes; here one 1024-thread block keeps the right-hand side and iterate of every
// remaining level in LDS and runs pre-smoothing, residual, restriction, the dense solve on
// the coarsest level, prolongation and post-smoothing with block barriers in between.
// The steps are those of the per-level launches: the same Chebyshev coefficients, the same
// stencil tables and restriction weights, the coarse quadratic for the prolongation.
//
// Threads: four groups of 256, one per node class (vertex, horizontal edge, vertical edge,
// diagonal: the parities of the lattice coordinates), so the stencil of a wave is uniform;
// on a level of n <= 16 cells every class has at most 256 interior nodes, one per thread.
// Dirichlet nodes hold 0 in every vector (a restricted right-hand side vanishes there and
// the identity rows keep it so), so only interior nodes are stepped.  A smoothing level's
// vectors lie in LDS as even and odd column planes ([component][parity][row][column / 2]):
// the lanes of a wave (one class, consecutive nodes of a row) then read consecutive words,
// without the bank conflicts of the stride-2 row-major order.  The coarsest level keeps the
// row-major order of its dense inverse.  The stencil
// coefficients, inverse diagonal blocks and restriction weights are copied to LDS first:
// read from device memory at every step they cost a scalar-cache round trip per few
// neighbours.
#include "ctx.h"
#include "kernels.h"
#include "lattice.h"
#include "stencil.h"

namespace fsi {

namespace {

constexpr int kTailThreads = 1024, kTailGroup = kTailThreads / 4;

// LDS layout of a smoothing level of n cells: planes of n + 1 columns
struct TailGrid {
  int L, HW, N;   // lattice side 2n + 1, plane width, entries per component (2 L HW)
  __device__ int at(int I, int J) const { return ((I & 1) * L + J) * HW + (I >> 1); }
};
__device__ __forceinline__ TailGrid tail_grid(int n) {
  const int L = 2 * n + 1;
  return TailGrid{L, n + 1, 2 * L * (n + 1)};
}
// floor(v / 2) for the small offsets of the stencils (v >= -4)
__host__ __device__ constexpr int half_floor(int v) { return (v + 4) / 2 - 2; }

// interior node of class c (I parity c & 1, J parity c >> 1) number i on a level of n cells
__device__ __forceinline__ bool class_node(int c, int i, int n, int &I, int &J) {
  const int pi = c & 1, pj = c >> 1;
  const int ni = pi ? n : n - 1, nj = pj ? n : n - 1;
  if (i >= ni * nj) return false;
  I = (pi ? 1 : 2) + 2 * (i % ni);
  J = (pj ? 1 : 2) + 2 * (i / ni);
  return true;
}

// (A_f x) at the node of LDS index idx (layout g); cf: the level's coefficients in LDS
// (class CLS at kTailCoef[CLS], four per entry).  A neighbour (dI, dJ) of a node of column
// parity P lies in plane (P + dI) mod 2, floor((P + dI) / 2) columns over.
template <typename T, int CLS>
__device__ __forceinline__ void tail_product(const T *cf, const T *x, const TailGrid &g, int idx, T &s0, T &s1) {
  constexpr StencilOffsets so = stencil_offsets();
  constexpr CrossZero cz = cross_zero();
  constexpr int P = CLS & 1;
  const int N = g.N;
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int k = 0; k < kStencilCount[CLS]; ++k) {
    const int dI = so.d[CLS][k][0], dJ = so.d[CLS][k][1];
    const int o = idx + ((((P + dI) & 1) - P) * g.L + dJ) * g.HW + half_floor(P + dI);
    const T y0 = x[o], y1 = x[N + o];
    const T *ck = cf + kTailCoef[CLS] + 4 * k;
    const T c0 = ck[0], c1 = ck[1], c2 = ck[2], c3 = ck[3];
    if (cz.z[CLS][k]) {
      s0 = fma(c0, y0, s0);
      s1 = fma(c3, y1, s1);
    } else {
      s0 = fma(c1, y1, fma(c0, y0, s0));
      s1 = fma(c3, y1, fma(c2, y0, s1));
    }
  }
}

template <typename T>
__device__ __forceinline__ void class_product(int c, const T *cf, const T *x, const TailGrid &g, int idx, T &s0,
                                              T &s1) {
  switch (c) {   // uniform over the wave
    case 0: tail_product<T, 0>(cf, x, g, idx, s0, s1); break;
    case 1: tail_product<T, 1>(cf, x, g, idx, s0, s1); break;
    case 2: tail_product<T, 2>(cf, x, g, idx, s0, s1); break;
    default: tail_product<T, 3>(cf, x, g, idx, s0, s1); break;
  }
}

// restriction sum at coarse node (Ic, Jc) of class CLS from the fine residual r (weights
// rw in LDS, class CLS at kTailRs[CLS])
template <typename T, int CLS>
__device__ __forceinline__ void tail_restrict(const T *rw, const T *r, const TailGrid &g, int Ic, int Jc, T &s0,
                                              T &s1) {
  constexpr RestrOffsets ro = restrict_offsets();
  const int N = g.N;
  s0 = 0;
  s1 = 0;
  const int c = 2 * Jc * g.HW + Ic;   // fine (2 Ic, 2 Jc): even plane
#pragma unroll
  for (int k = 0; k < kRestrCount[CLS]; ++k) {
    const int dI = ro.d[CLS][k][0], dJ = ro.d[CLS][k][1];
    const int o = c + ((dI & 1) * g.L + dJ) * g.HW + half_floor(dI);
    const T w = rw[kTailRs[CLS] + k];
    s0 = fma(w, r[o], s0);
    s1 = fma(w, r[N + o], s1);
  }
}

// coarse quadratic at fine node (I, J): the six P2 basis values of the coarse cell's
// triangle at the local position, in the order vertices 0, 1, 2, edges 01, 12, 20 (exact in
// float).  The coarse vector xc is a smoothing level (layout gc) or, when natural, the
// coarsest level in row-major order (side gc.L, gc.N nodes per component).
template <typename T>
__device__ __forceinline__ void tail_prolong(const T *xc, const TailGrid &gc, bool natural, int I, int J, T &s0,
                                             T &s1) {
  const int A = I & 3, B = J & 3, Ib = 2 * (I >> 2), Jb = 2 * (J >> 2);
  const bool lo = A >= B;
  const float xi = 0.25f * (float)A, eta = 0.25f * (float)B;
  const float l0 = lo ? 1.0f - xi : 1.0f - eta, l1 = lo ? xi - eta : xi, l2 = lo ? eta : eta - xi;
  const float phi[6] = {l0 * (2.0f * l0 - 1.0f), l1 * (2.0f * l1 - 1.0f), l2 * (2.0f * l2 - 1.0f),
                        4.0f * l0 * l1,         4.0f * l1 * l2,         4.0f * l2 * l0};
  const int di[6] = {0, 2, lo ? 2 : 0, 1, lo ? 2 : 1, lo ? 1 : 0};
  const int dj[6] = {0, lo ? 0 : 2, 2, lo ? 0 : 1, lo ? 1 : 2, 1};
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const T w = (T)phi[q];
    const int Ic = Ib + di[q], Jc = Jb + dj[q];
    const int k = natural ? Jc * gc.L + Ic : gc.at(Ic, Jc);
    s0 = fma(w, xc[k], s0);
    s1 = fma(w, xc[gc.N + k], s1);
  }
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_mg_tail(TailArgs<T> a) {
  extern __shared__ unsigned char tail_smem[];
  T *sm = reinterpret_cast<T *>(tail_smem);
  // the class group is uniform over a wave: scalar branches and scalar table loads
  const int tid = threadIdx.x, grp = __builtin_amdgcn_readfirstlane(tid / kTailGroup), gi = tid % kTailGroup;
  const T *bg = a.b + (int64_t)blockIdx.y * a.lb;
  T *xg = a.x + (int64_t)blockIdx.y * a.lb;
  // device-memory operands of the start issued first, so that their latency overlaps the
  // clearing of the vectors and the table copies: the dense inverse (when it goes to LDS,
  // kPre entries per thread at once) and the first level's right-hand side (stored after
  // the clearing barrier)
  constexpr int kPre = 12;
  const int mm = a.offm >= 0 ? a.m * a.m : 0;
  T pre[kPre];
#pragma unroll
  for (int q = 0; q < kPre; ++q) {
    const int i = tid + kTailThreads * q;
    pre[q] = i < mm ? a.cinv[i] : T(0);
  }
  T b0v = 0, b1v = 0;
  int bk = -1;
  {
    const TailGrid g = tail_grid(a.lv[0].n);
    const int NG = g.L * g.L;   // nodes per component in device memory (row-major)
    int I, J;
    if (class_node(grp, gi, a.lv[0].n, I, J)) {
      const int kg = J * g.L + I;
      bk = g.at(I, J);
      b0v = bg[kg];
      b1v = bg[NG + kg];
    }
  }
  for (int i = tid; i < a.offt; i += kTailThreads) sm[i] = T(0);
  for (int l = 0; l < a.nlev; ++l)   // coefficients (class-compact) and inverse diagonal blocks
    for (int i = tid; i < kTailTab; i += kTailThreads) {
      const StencilTable<T> &tb = *a.lv[l].tab;
      T v;
      if (i >= kTailCoef[3] + 4 * kStencilCount[3]) {
        const int j = i - (kTailCoef[3] + 4 * kStencilCount[3]);
        v = tb.dinv[j / 4][j % 4];
      } else {
        const int c = i < kTailCoef[1] ? 0 : i < kTailCoef[2] ? 1 : i < kTailCoef[3] ? 2 : 3;
        const int j = i - kTailCoef[c];
        v = tb.coef[c][j / 4][j % 4];
      }
      sm[a.offt + l * kTailTab + i] = v;
    }
  for (int i = tid; i < kTailRw; i += kTailThreads) {
    const int c = i < kTailRs[1] ? 0 : i < kTailRs[2] ? 1 : i < kTailRs[3] ? 2 : 3;
    sm[a.offt + a.nlev * kTailTab + i] = a.rt->w[c][i - kTailRs[c]];
  }
#pragma unroll
  for (int q = 0; q < kPre; ++q) {
    const int i = tid + kTailThreads * q;
    if (i < mm) sm[a.offm + i] = pre[q];
  }
  for (int i = tid + kTailThreads * kPre; i < mm; i += kTailThreads) sm[a.offm + i] = a.cinv[i];
  __syncthreads();
  const T *rw = sm + a.offt + a.nlev * kTailTab;
  auto coefs = [&](int l) { return (const T *)(sm + a.offt + l * kTailTab); };
  auto dinv = [&](int l) { return (const T *)(sm + a.offt + l * kTailTab + kTailCoef[3] + 4 * kStencilCount[3]); };
  T *d = sm + a.offd;   // the direction (then residual) of the level being smoothed
  if (bk >= 0) {        // right-hand side of the first level (interior nodes)
    T *b = sm + a.lv[0].off;
    b[bk] = b0v;
    b[tail_grid(a.lv[0].n).N + bk] = b1v;
  }
  __syncthreads();
  // one Chebyshev step on level l from x (first: c1 = 0, the direction is not read)
  auto cheb_step = [&](int l, bool first, T c1, T c2) {
    const TailLevel<T> &lv = a.lv[l];
    const TailGrid g = tail_grid(lv.n);
    const int N = g.N;
    T *b = sm + lv.off, *x = b + 2 * N;
    int I, J;
    const bool mine = class_node(grp, gi, lv.n, I, J);
    const int k = mine ? g.at(I, J) : 0;
    T x0 = 0, x1 = 0, d0 = 0, d1 = 0;
    if (mine) {
      T s0, s1;
      class_product<T>(grp, coefs(l), x, g, k, s0, s1);
      const T r0 = b[k] - s0, r1 = b[N + k] - s1;
      const T *di = dinv(l) + 4 * grp;
      const T z0 = di[0] * r0 + di[1] * r1, z1 = di[2] * r0 + di[3] * r1;
      d0 = first ? c2 * z0 : c1 * d[k] + c2 * z0;
      d1 = first ? c2 * z1 : c1 * d[N + k] + c2 * z1;
      x0 = x[k] + d0;
      x1 = x[N + k] + d1;
    }
    __syncthreads();
    if (mine) {
      x[k] = x0;
      x[N + k] = x1;
      d[k] = d0;
      d[N + k] = d1;
    }
    __syncthreads();
  };
  // descent: pre-smoothing, residual, restriction
  for (int l = 0; l < a.nlev; ++l) {
    const TailLevel<T> &lv = a.lv[l];
    const TailGrid g = tail_grid(lv.n);
    const int N = g.N;
    T *b = sm + lv.off, *x = b + 2 * N;
    {   // first step from zero: x = d = s D^{-1} b
      int I, J;
      if (class_node(grp, gi, lv.n, I, J)) {
        const int k = g.at(I, J);
        const T *di = dinv(l) + 4 * grp;
        const T b0 = b[k], b1 = b[N + k];
        const T z0 = lv.s * (di[0] * b0 + di[1] * b1), z1 = lv.s * (di[2] * b0 + di[3] * b1);
        x[k] = d[k] = z0;
        x[N + k] = d[N + k] = z1;
      }
    }
    __syncthreads();
    for (int j = 0; j + 1 < a.degree; ++j) cheb_step(l, false, lv.c1[j], lv.c2[j]);
    {   // residual over the direction (not read again before the post-smoothing)
      int I, J;
      if (class_node(grp, gi, lv.n, I, J)) {
        const int k = g.at(I, J);
        T s0, s1;
        class_product<T>(grp, coefs(l), x, g, k, s0, s1);
        d[k] = b[k] - s0;
        d[N + k] = b[N + k] - s1;
      }
    }
    __syncthreads();
    {   // restriction into the next level's right-hand side (interior coarse nodes)
      const int nc = lv.n / 2, Lc = lv.n + 1;
      const bool coarsest = l + 1 == a.nlev;   // row-major, as its dense inverse
      const TailGrid gc = coarsest ? TailGrid{Lc, 0, Lc * Lc} : tail_grid(nc);
      T *bc = coarsest ? sm + a.offc : sm + a.lv[l + 1].off;
      int Ic, Jc;
      if (class_node(grp, gi, nc, Ic, Jc)) {
        const int k = coarsest ? Jc * Lc + Ic : gc.at(Ic, Jc);
        T s0, s1;
        switch (grp) {
          case 0: tail_restrict<T, 0>(rw, d, g, Ic, Jc, s0, s1); break;
          case 1: tail_restrict<T, 1>(rw, d, g, Ic, Jc, s0, s1); break;
          case 2: tail_restrict<T, 2>(rw, d, g, Ic, Jc, s0, s1); break;
          default: tail_restrict<T, 3>(rw, d, g, Ic, Jc, s0, s1); break;
        }
        bc[k] = s0;
        bc[gc.N + k] = s1;
      }
    }
    __syncthreads();
  }
  {   // coarsest level: x = C^{-1} b, one wave per row (sums in double, as the dense kernel);
      // a wave loads kRows rows at once (coalesced, one memory round trip per batch), from
      // LDS when the inverse was copied there
    constexpr int kRows = 4, kSeg = kTailDenseMax / kWave, NW = kTailThreads / kWave;
    const T *b = sm + a.offc;
    T *x = sm + a.offc + a.m;
    const int w = tid / kWave, lane = tid % kWave;
    auto dense = [&](const T *cm) {
      for (int r0 = w; r0 < a.m; r0 += kRows * NW) {
        T c[kRows][kSeg];
#pragma unroll
        for (int q = 0; q < kRows; ++q)
#pragma unroll
          for (int j = 0; j < kSeg; ++j) {
            const int r = r0 + q * NW, k = lane + kWave * j;
            c[q][j] = (r < a.m && k < a.m) ? cm[(int64_t)r * a.m + k] : T(0);
          }
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < kSeg; ++j)
            if (lane + kWave * j < a.m) s += (double)c[q][j] * (double)b[lane + kWave * j];
          s = wave_sum(s);
          if (lane == 0 && r0 + q * NW < a.m) x[r0 + q * NW] = (T)s;
        }
      }
    };
    if (a.offm >= 0) dense(sm + a.offm);
    else dense(a.cinv);
  }
  __syncthreads();
  // ascent: coarse correction, post-smoothing
  for (int l = a.nlev - 1; l >= 0; --l) {
    const TailLevel<T> &lv = a.lv[l];
    const TailGrid g = tail_grid(lv.n);
    const int N = g.N;
    T *b = sm + lv.off, *x = b + 2 * N;
    const int Lc = lv.n + 1;
    const bool coarsest = l + 1 == a.nlev;
    const TailGrid gc = coarsest ? TailGrid{Lc, 0, Lc * Lc} : tail_grid(lv.n / 2);
    const T *xc = coarsest ? sm + a.offc + a.m : sm + a.lv[l + 1].off + 2 * gc.N;
    int I, J;
    if (class_node(grp, gi, lv.n, I, J)) {
      const int k = g.at(I, J);
      T s0, s1;
      tail_prolong<T>(xc, gc, coarsest, I, J, s0, s1);
      x[k] += s0;
      x[N + k] += s1;
    }
    __syncthreads();
    cheb_step(l, true, T(0), lv.s);
    for (int j = 0; j + 1 < a.degree; ++j) cheb_step(l, false, lv.c1[j], lv.c2[j]);
    (void)b;
  }
  {   // result of the first level in row-major order, Dirichlet nodes included (0)
    const TailGrid g = tail_grid(a.lv[0].n);
    const int NG = g.L * g.L;
    const T *x = sm + a.lv[0].off + 2 * g.N;
    for (int i = tid; i < NG; i += kTailThreads) {
      const int k = g.at(i % g.L, i / g.L);
      xg[i] = x[k];
      xg[NG + i] = x[g.N + k];
    }
  }
}

// ---------------------------------------------------------------- pressure (P1) tail
// The coarse end of the Cahouet-Chabard Laplacian V-cycle: on levels of at most 64 x 64
// cells the per-level launches (smoothing, residual, restriction, prolongation) cost the
// latency of a kernel each for a few thousand nodes.  One 1024-thread block keeps every
// remaining level in LDS and runs the steps of those launches with block barriers between
// passes: the Chebyshev steps of k_p1_multi (same coefficients, same order of the stencil
// sums, the pinned row and column), the residual of k_p1, the restriction of k_p1_restrict,
// the dense coarsest solve of k_dense_mv and the linear prolongation of k_p1_prolong_add.
// Node r of a level belongs to thread r mod 1024 in every pass, so its search direction stays
// in that thread's registers.

// (A x)_r on a P1 level of n cells (row-major x, side L = n + 1), as k_p1 sums it
template <typename T>
__device__ __forceinline__ T p1_apply(const T *tb, int pin, const T *x, int n, int r) {
  const int L = n + 1, i = r % L, j = r / L;
  const T xc = x[r];
  if (pin && r == 0) return xc;   // identity row of the pinned node
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  const T *c = tb + kP1Nbr * (3 * cj + ci);
  // column 0 is zero when pinned: node (0, 0) is read as 0
  auto ld = [&](int q) -> T { return (pin && q == 0) ? T(0) : x[q]; };
  T s = c[0] * xc;
  if (i > 0) s += c[1] * ld(r - 1);
  if (i < n) s += c[2] * x[r + 1];
  if (j > 0) s += c[3] * ld(r - L);
  if (j < n) s += c[4] * x[r + L];
  if (i > 0 && j > 0) s += c[5] * ld(r - L - 1);
  if (i < n && j < n) s += c[6] * x[r + L + 1];
  return s;
}

template <typename T>
__device__ __forceinline__ T p1_dinv(const T *tb, int n, int r) {
  const int L = n + 1, i = r % L, j = r / L;
  const int ci = i == 0 ? 0 : (i == n ? 2 : 1), cj = j == 0 ? 0 : (j == n ? 2 : 1);
  return tb[9 * kP1Nbr + 3 * cj + ci];
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_p1_tail(PTailArgs<T> a) {
  extern __shared__ unsigned char ptail_smem[];
  T *sm = reinterpret_cast<T *>(ptail_smem);
  const int tid = threadIdx.x;
  const T *bg = a.b + (int64_t)blockIdx.y * a.lb;
  T *xg = a.x + (int64_t)blockIdx.y * a.lb;
  {   // the first level's right-hand side, the tables, the dense inverse (when in LDS)
    const int L0 = a.lv[0].n + 1, N0 = L0 * L0;
    for (int r = tid; r < N0; r += kTailThreads) sm[a.lv[0].off + r] = bg[r];
    for (int l = 0; l < a.nlev; ++l)
      for (int i = tid; i < kPTailTab; i += kTailThreads) {
        const P1Table<T> &tb = *a.lv[l].tab;
        sm[a.offt + l * kPTailTab + i] = i < 9 * kP1Nbr ? tb.coef[i / kP1Nbr][i % kP1Nbr] : tb.dinv[i - 9 * kP1Nbr];
      }
    if (a.offm >= 0)
      for (int i = tid; i < a.m * a.m; i += kTailThreads) sm[a.offm + i] = a.cinv[i];
  }
  __syncthreads();
  T *x2 = sm + a.offx2;
  T dreg[kPTailPer];
  // S Chebyshev steps on level l from zero (ZERO) or from its x; the result ends in x
  auto smooth = [&](int l, bool zero) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, N = (n + 1) * (n + 1);
    const T *tb = sm + a.offt + l * kPTailTab;
    const int pin = lv.tab->pin;
    T *b = sm + lv.off, *x = b + N;
    int k0 = 0;
    if (zero) {   // x = d = c2[0] D^{-1} b
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) {
        const int r = tid + kTailThreads * q;
        if (r < N) {
          const T z = lv.c2[0] * (p1_dinv(tb, n, r) * b[r]);
          dreg[q] = z;
          x[r] = z;
        }
      }
      k0 = 1;
      __syncthreads();
    } else {
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) dreg[q] = T(0);
    }
    T *src = x, *dst = x2;
    for (int k = k0; k < a.degree; ++k) {
#pragma unroll
      for (int q = 0; q < kPTailPer; ++q) {
        const int r = tid + kTailThreads * q;
        if (r < N) {
          const T sum = p1_apply(tb, pin, src, n, r);
          const T z = p1_dinv(tb, n, r) * (b[r] - sum);
          const T dn = lv.c1[k] * dreg[q] + lv.c2[k] * z;
          dreg[q] = dn;
          dst[r] = src[r] + dn;
        }
      }
      __syncthreads();
      T *t = src;
      src = dst;
      dst = t;
    }
    if (src != x) {   // an odd number of steps from x left the result in the second buffer
      for (int r = tid; r < N; r += kTailThreads) x[r] = src[r];
      __syncthreads();
    }
  };
  // descent: pre-smoothing, residual (into the second buffer), restriction
  for (int l = 0; l < a.nlev; ++l) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, L = n + 1, N = L * L;
    const T *tb = sm + a.offt + l * kPTailTab;
    T *b = sm + lv.off, *x = b + N;
    smooth(l, true);
    const int pin = lv.tab->pin;
    for (int r = tid; r < N; r += kTailThreads) x2[r] = b[r] - p1_apply(tb, pin, x, n, r);
    __syncthreads();
    const int nc = n / 2, Lc = nc + 1;
    const bool coarsest = l + 1 == a.nlev;
    T *bc = coarsest ? sm + a.offc : sm + a.lv[l + 1].off;
    for (int q = tid; q < Lc * Lc; q += kTailThreads) {
      if (q == 0) {
        bc[0] = T(0);
        continue;
      }
      const int fi = 2 * (q % Lc), fj = 2 * (q / Lc);
      auto fv = [&](int u, int v) -> T {
        if (u < 0 || v < 0 || u > n || v > n) return T(0);
        const int f = v * L + u;
        return f == 0 ? T(0) : x2[f];
      };
      const T edges = fv(fi - 1, fj) + fv(fi + 1, fj) + fv(fi, fj - 1) + fv(fi, fj + 1) + fv(fi + 1, fj + 1) +
                      fv(fi - 1, fj - 1);
      bc[q] = fv(fi, fj) + T(0.5) * edges;
    }
    __syncthreads();
  }
  {   // coarsest level: x = C^{-1} b, one wave per row, sums in double (as k_dense_mv)
    const T *b = sm + a.offc;
    T *x = sm + a.offc + a.m;
    const T *cm = a.offm >= 0 ? sm + a.offm : a.cinv;
    const int w = tid / kWave, lane = tid % kWave;
    for (int r = w; r < a.m; r += kTailThreads / kWave) {
      double s = 0.0;
      for (int k = lane; k < a.m; k += kWave) s += (double)cm[(int64_t)r * a.m + k] * (double)b[k];
      s = wave_sum(s);
      if (lane == 0) x[r] = (T)s;
    }
  }
  __syncthreads();
  // ascent: linear prolongation of the coarse correction (the pinned node excluded), post-smoothing
  for (int l = a.nlev - 1; l >= 0; --l) {
    const PTailLevel<T> &lv = a.lv[l];
    const int n = lv.n, L = n + 1, N = L * L, Lc = n / 2 + 1;
    T *x = sm + lv.off + N;
    const T *xc = l + 1 == a.nlev ? sm + a.offc + a.m : sm + a.lv[l + 1].off + Lc * Lc;
    for (int r = tid; r < N; r += kTailThreads) {
      if (r == 0) continue;
      const int i = r % L, j = r / L, ci = i >> 1, cj = j >> 1;
      auto cv = [&](int u, int v) -> T {
        const int k = v * Lc + u;
        return k == 0 ? T(0) : xc[k];
      };
      T s;
      if (!(i & 1) && !(j & 1)) s = cv(ci, cj);
      else if (!(j & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj);
      else if (!(i & 1)) s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci, cj + 1);
      else s = T(0.5) * cv(ci, cj) + T(0.5) * cv(ci + 1, cj + 1);
      x[r] += s;
    }
    __syncthreads();
    smooth(l, false);
  }
  {
    const int N0 = (a.lv[0].n + 1) * (a.lv[0].n + 1);
    const T *x = sm + a.lv[0].off + N0;
    for (int r = tid; r < N0; r += kTailThreads) xg[r] = x[r];
  }
}

}  // namespace

int tail_lds_limit() {
  static int limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    v = v < 65536 ? v : v > 163840 ? 163840 : v;
    // dynamic LDS above 64 KiB is granted per kernel
    if (v > 65536 && (hipFuncSetAttribute((const void *)k_mg_tail<double>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess ||
                      hipFuncSetAttribute((const void *)k_mg_tail<float>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess ||
                      hipFuncSetAttribute((const void *)k_p1_tail<double>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess ||
                      hipFuncSetAttribute((const void *)k_p1_tail<float>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess)) {
      (void)hipGetLastError();
      v = 65536;
    }
    return v;
  }();
  return limit;
}

template <typename T>
void mg_tail(const TailArgs<T> &a, hipStream_t s, int K) {
  FSI_REQUIRE(a.nlev >= 1 && a.nlev <= kTailMax && a.degree >= 1 && a.degree <= kTailDeg, FSI_E_ARG,
              "coarse tail shape out of range");
  FSI_REQUIRE(a.lv[0].n <= kTailMaxN, FSI_E_ARG, "coarse tail level too fine");
  FSI_REQUIRE(a.m <= kTailDenseMax, FSI_E_ARG, "coarsest level too large for the tail");
  FSI_REQUIRE(K >= 1 && K <= 65535 && (K == 1 || a.lb > 0), FSI_E_ARG, "lane count out of range");
  const int bytes = a.lds * (int)sizeof(T);
  FSI_REQUIRE(bytes <= tail_lds_limit(), FSI_E_ARG, "coarse tail exceeds the LDS of a block");
  hipLaunchKernelGGL(k_mg_tail<T>, dim3(1, (unsigned)K), dim3(kTailThreads), bytes, s, a);
  FSI_CHECK_LAUNCH();
}
template void mg_tail<double>(const TailArgs<double> &, hipStream_t, int);
template void mg_tail<float>(const TailArgs<float> &, hipStream_t, int);

template <typename T>
void p1_tail(const PTailArgs<T> &a, hipStream_t s, int K) {
  FSI_REQUIRE(a.nlev >= 1 && a.nlev <= kPTailMax && a.degree >= 1 && a.degree <= kPTailDeg, FSI_E_ARG,
              "pressure tail shape out of range");
  FSI_REQUIRE(a.lv[0].n <= kPTailMaxN && (a.lv[0].n + 1) * (a.lv[0].n + 1) <= kPTailPer * kTailThreads, FSI_E_ARG,
              "pressure tail level too fine");
  for (int l = 0; l + 1 < a.nlev; ++l)
    FSI_REQUIRE(a.lv[l + 1].n * 2 == a.lv[l].n, FSI_E_ARG, "pressure tail levels not nested");
  FSI_REQUIRE(a.m == (a.lv[a.nlev - 1].n / 2 + 1) * (a.lv[a.nlev - 1].n / 2 + 1) && a.m <= kPTailDenseMax, FSI_E_ARG,
              "pressure tail coarsest level out of range");
  FSI_REQUIRE(K >= 1 && K <= 65535 && (K == 1 || a.lb > 0), FSI_E_ARG, "lane count out of range");
  const int bytes = a.lds * (int)sizeof(T);
  FSI_REQUIRE(bytes <= tail_lds_limit(), FSI_E_ARG, "pressure tail exceeds the LDS of a block");
  hipLaunchKernelGGL(k_p1_tail<T>, dim3(1, (unsigned)K), dim3(kTailThreads), bytes, s, a);
  FSI_CHECK_LAUNCH();
}
template void p1_tail<double>(const PTailArgs<double> &, hipStream_t, int);
template void p1_tail<float>(const PTailArgs<float> &, hipStream_t, int);

}  // namespace fsi
