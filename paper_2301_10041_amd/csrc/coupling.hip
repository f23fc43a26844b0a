// C_f(X^n) on the device (Sec. 4, the coupling assembly after eq. (matrix)):
//   (C_f)_lj = sum_E (|E| / |X^n(E)|) int_{X^n(E)} lam_l(x) phi_j(x) dx,
// where X^n is affine on each solid triangle E, lam_l are the barycentric coordinates of
// the mapped triangle and phi_j the P2 fluid basis.  The paper finds the fluid elements
// met by X^n(E) through its bounding box on the Cartesian grid and clips with the
// Sutherland-Hodgman algorithm; each piece is integrated exactly.
//
// Pipeline (all on the stream, no floating-point atomics):
//   1. per solid triangle: validity (area > 0, inside [0,1]^2) and candidate cell count
//   2. scan -> candidate offsets
//   3. per candidate cell: clip, count kept pieces (fluid triangles T0/T1 of the cell)
//   4. scan -> piece offsets
//   5. per candidate cell: clip again, write (E, T) and the 3x6 local matrix of each piece
//   6. per solid node (one wavefront): rows of C_f with a window bitmap in LDS (columns in
//      ascending order), values summed in a fixed order
//   7. C_f^T: counting transpose, then each entry moved to its rank in its row (deterministic)
//
// Clipping arithmetic (must be reproduced bit for bit wherever the intersection list is
// compared): clip against x >= x_i, x <= x_{i+1}, y >= y_j, y <= y_{j+1}, then against
// (x - x_i) - (y - y_j) >= 0 (T0) or (y - y_j) - (x - x_i) >= 0 (T1); keep a vertex if its
// value is >= 0, emit a crossing a + t (b - a), t = f_a / (f_a - f_b), only for strictly
// opposite signs, with the axis coordinate set to the line value; keep a piece iff its fan
// area from vertex 0 exceeds 5e-11 h^2.  This file is compiled with -ffp-contract=off so
// that no product is fused into an addition.
#include <cmath>
#include <mutex>
#include <string>

#include "ctx.h"
#include "kernels.h"

namespace fsi {

constexpr int kMaxPoly = 12;       // a triangle clipped by 5 half-planes has <= 8 vertices
constexpr int kWinCap = 4096;      // LDS window of P2 nodes per C_f row (64 x 64); larger ones in device memory

enum { DF_MESH = 1 };

struct Pt {
  double x, y;
};

__device__ __forceinline__ void load_tri(const double *X, int64_t ns, const int *tri, int e, Pt *P) {
  for (int m = 0; m < 3; ++m) {
    int v = tri[3 * e + m];
    P[m].x = X[v];
    P[m].y = X[ns + v];
  }
}

__device__ __forceinline__ double tri_area(const Pt *P) {
  return 0.5 * ((P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[2].x - P[0].x) * (P[1].y - P[0].y));
}

__device__ __forceinline__ void cell_range(const Pt *P, int n, int &i0, int &i1, int &j0, int &j1) {
  double xmin = fmin(fmin(P[0].x, P[1].x), P[2].x), xmax = fmax(fmax(P[0].x, P[1].x), P[2].x);
  double ymin = fmin(fmin(P[0].y, P[1].y), P[2].y), ymax = fmax(fmax(P[0].y, P[1].y), P[2].y);
  double dn = (double)n;
  i0 = (int)floor(xmin * dn);
  i1 = (int)floor(xmax * dn);
  j0 = (int)floor(ymin * dn);
  j1 = (int)floor(ymax * dn);
  i0 = min(max(i0, 0), n - 1);
  i1 = min(max(i1, 0), n - 1);
  j0 = min(max(j0, 0), n - 1);
  j1 = min(max(j1, 0), n - 1);
}

// keep coord(axis) >= c (ge) or <= c
__device__ __forceinline__ int clip_axis(const Pt *in, int m, Pt *out, int axis, double c, bool ge) {
  int k = 0;
  for (int q = 0; q < m; ++q) {
    Pt a = in[q], b = in[(q + 1) % m];
    double av = axis ? a.y : a.x, bv = axis ? b.y : b.x;
    double fa = ge ? (av - c) : (c - av);
    double fb = ge ? (bv - c) : (c - bv);
    if (fa >= 0.0) out[k++] = a;
    if ((fa > 0.0 && fb < 0.0) || (fa < 0.0 && fb > 0.0)) {
      double t = fa / (fa - fb);
      if (axis == 0) out[k++] = Pt{c, a.y + t * (b.y - a.y)};
      else out[k++] = Pt{a.x + t * (b.x - a.x), c};
    }
  }
  return k;
}

__device__ __forceinline__ int clip_diag(const Pt *in, int m, Pt *out, double xi, double yj, bool upper) {
  int k = 0;
  for (int q = 0; q < m; ++q) {
    Pt a = in[q], b = in[(q + 1) % m];
    double fa, fb;
    if (upper) {
      fa = (a.y - yj) - (a.x - xi);
      fb = (b.y - yj) - (b.x - xi);
    } else {
      fa = (a.x - xi) - (a.y - yj);
      fb = (b.x - xi) - (b.y - yj);
    }
    if (fa >= 0.0) out[k++] = a;
    if ((fa > 0.0 && fb < 0.0) || (fa < 0.0 && fb > 0.0)) {
      double t = fa / (fa - fb);
      out[k++] = Pt{a.x + t * (b.x - a.x), a.y + t * (b.y - a.y)};
    }
  }
  return k;
}

__device__ __forceinline__ double fan_area(const Pt *p, int m) {
  if (m < 3) return 0.0;
  double s = 0.0;
  for (int k = 1; k < m - 1; ++k)
    s += (p[k].x - p[0].x) * (p[k + 1].y - p[0].y) - (p[k + 1].x - p[0].x) * (p[k].y - p[0].y);
  return 0.5 * s;
}

// Square clip of the mapped triangle with cell (i, j); returns the vertex count in sq.
__device__ __forceinline__ int clip_cell(const Pt *P, int n, int i, int j, Pt *sq) {
  Pt a[kMaxPoly], b[kMaxPoly];
  double dn = (double)n;
  double xi = (double)i / dn, xi1 = (double)(i + 1) / dn;
  double yj = (double)j / dn, yj1 = (double)(j + 1) / dn;
  int m = clip_axis(P, 3, a, 0, xi, true);
  m = clip_axis(a, m, b, 0, xi1, false);
  m = clip_axis(b, m, a, 1, yj, true);
  m = clip_axis(a, m, sq, 1, yj1, false);
  return m;
}

// bit t set iff the piece with fluid triangle t of cell (i, j) is kept; the pieces are
// returned in q[t] / mq[t].
__device__ __forceinline__ int clip_pieces(const Pt *P, int n, int i, int j, Pt q[2][kMaxPoly], int mq[2]) {
  Pt sq[kMaxPoly];
  int m = clip_cell(P, n, i, j, sq);
  int mask = 0;
  mq[0] = mq[1] = 0;
  if (m < 3) return 0;
  double dn = (double)n;
  double xi = (double)i / dn, yj = (double)j / dn;
  double h = 1.0 / dn;
  double tau = 5e-11 * h * h;
  for (int t = 0; t < 2; ++t) {
    int k = clip_diag(sq, m, q[t], xi, yj, t == 1);
    if (k >= 3 && fan_area(q[t], k) > tau) {
      mask |= 1 << t;
      mq[t] = k;
    }
  }
  return mask;
}

__global__ void k_cand_count(int64_t nt, int64_t ns, int n, const double *__restrict__ X,
                             const int *__restrict__ tri, int *cnt, int *flag) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  Pt P[3];
  load_tri(X, ns, tri, (int)e, P);
  bool ok = tri_area(P) > 0.0;
  for (int m = 0; m < 3; ++m)
    ok = ok && P[m].x >= 0.0 && P[m].x <= 1.0 && P[m].y >= 0.0 && P[m].y <= 1.0;
  if (!ok) {
    atomicOr(flag, DF_MESH);
    cnt[e] = 0;
    return;
  }
  int i0, i1, j0, j1;
  cell_range(P, n, i0, i1, j0, j1);
  cnt[e] = (i1 - i0 + 1) * (j1 - j0 + 1);
}

__device__ __forceinline__ int find_owner(const int *off, int64_t nt, int64_t c) {
  // largest e with off[e] <= c  (off is non-decreasing, off[0] = 0)
  int64_t lo = 0, hi = nt;   // answer in [0, nt)
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= c) lo = mid;
    else hi = mid;
  }
  return (int)lo;
}

__device__ __forceinline__ void cand_cell(const Pt *P, int n, int q, int &i, int &j) {
  int i0, i1, j0, j1;
  cell_range(P, n, i0, i1, j0, j1);
  int w = i1 - i0 + 1;
  i = i0 + q % w;
  j = j0 + q / w;
}

__global__ void k_clip_count(int64_t ncand, int64_t nt, int64_t ns, int n, const double *__restrict__ X,
                             const int *__restrict__ tri, const int *__restrict__ cand_off,
                             int *piece_cnt) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncand) return;
  int e = find_owner(cand_off, nt, c);
  Pt P[3];
  load_tri(X, ns, tri, e, P);
  int i, j;
  cand_cell(P, n, (int)(c - cand_off[e]), i, j);
  Pt q[2][kMaxPoly];
  int mq[2];
  int mask = clip_pieces(P, n, i, j, q, mq);
  piece_cnt[c] = (mask & 1) + ((mask >> 1) & 1);
}

// Degree-4 six-point rule (Dunavant) on each fan triangle: exact for the cubic
// integrand lam_l * phi_j.
__constant__ double kQa[2] = {0.445948490915965, 0.091576213509771};
__constant__ double kQw[2] = {0.223381589678011, 0.109951743655322};

__device__ void piece_matrix(const Pt *P, const Pt *q, int m, int i, int j, int t, int n,
                             double ratio, double *L) {
  double acc[18];
  for (int k = 0; k < 18; ++k) acc[k] = 0.0;
  double D = (P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[2].x - P[0].x) * (P[1].y - P[0].y);
  double dn = (double)n;
  double xi0 = (double)i / dn, yj0 = (double)j / dn;
  for (int k = 1; k < m - 1; ++k) {
    Pt A = q[0], B = q[k], C = q[k + 1];
    double a2 = 0.5 * ((B.x - A.x) * (C.y - A.y) - (C.x - A.x) * (B.y - A.y));
    for (int g = 0; g < 6; ++g) {
      int grp = g / 3, rot = g % 3;
      double la = kQa[grp], lb = 1.0 - 2.0 * la;
      double l[3];
      l[rot] = lb; l[(rot + 1) % 3] = la; l[(rot + 2) % 3] = la;
      double w = kQw[grp] * a2;
      double x = l[0] * A.x + l[1] * B.x + l[2] * C.x;
      double y = l[0] * A.y + l[1] * B.y + l[2] * C.y;
      // barycentric coordinates in the mapped solid triangle
      double lam[3];
      lam[0] = ((P[1].x - x) * (P[2].y - y) - (P[2].x - x) * (P[1].y - y)) / D;
      lam[1] = ((P[2].x - x) * (P[0].y - y) - (P[0].x - x) * (P[2].y - y)) / D;
      lam[2] = 1.0 - lam[0] - lam[1];
      // P2 basis on the fluid triangle (local coordinates of the cell)
      double xs = (x - xi0) * dn, ys = (y - yj0) * dn;
      double mu[3];
      if (t == 0) { mu[0] = 1.0 - xs; mu[1] = xs - ys; mu[2] = ys; }
      else { mu[0] = 1.0 - ys; mu[1] = xs; mu[2] = ys - xs; }
      double phi[6] = {mu[0] * (2 * mu[0] - 1), mu[1] * (2 * mu[1] - 1), mu[2] * (2 * mu[2] - 1),
                       4 * mu[0] * mu[1], 4 * mu[1] * mu[2], 4 * mu[2] * mu[0]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 6; ++b) acc[a * 6 + b] += w * lam[a] * phi[b];
    }
  }
  for (int k = 0; k < 18; ++k) L[k] = ratio * acc[k];
}

__global__ void k_clip_emit(int64_t ncand, int64_t nt, int64_t ns, int n, const double *__restrict__ X,
                            const int *__restrict__ tri, const double *__restrict__ ref_area,
                            const int *__restrict__ cand_off, const int *__restrict__ piece_off,
                            int *pair_E, int *pair_T, double *piece_L) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncand) return;
  int e = find_owner(cand_off, nt, c);
  Pt P[3];
  load_tri(X, ns, tri, e, P);
  int i, j;
  cand_cell(P, n, (int)(c - cand_off[e]), i, j);
  Pt q[2][kMaxPoly];
  int mq[2];
  int mask = clip_pieces(P, n, i, j, q, mq);
  int p = piece_off[c];
  double ratio = ref_area[e] / tri_area(P);
  for (int t = 0; t < 2; ++t) {
    if (!(mask & (1 << t))) continue;
    pair_E[p] = e;
    pair_T[p] = 2 * (j * n + i) + t;
    piece_matrix(P, q[t], mq[t], i, j, t, n, ratio, piece_L + 18 * (int64_t)p);
    ++p;
  }
}

__global__ void k_elem_piece_off(int64_t nt, const int *cand_off, const int *piece_off, int *e_piece) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nt) return;
  e_piece[e] = piece_off[cand_off[e]];
}

// ---- rows of C_f: one wavefront per solid node
// Lattice offsets (x, y), in half cells from the cell's lower-left corner, of the six P2 nodes
// of fluid triangle t (vertices, then edge midpoints 01, 12, 20):
//   t = 0: (0,0) (2,0) (2,2) (1,0) (2,1) (1,1);  t = 1: (0,0) (2,2) (0,2) (1,1) (1,2) (0,1);
// packed two bits per node so that a runtime (t, b) costs shifts, not a table load.
constexpr unsigned pack6(int a0, int a1, int a2, int a3, int a4, int a5) {
  return (unsigned)(a0 | a1 << 2 | a2 << 4 | a3 << 6 | a4 << 8 | a5 << 10);
}
constexpr unsigned kOffX = pack6(0, 2, 2, 1, 2, 1) | pack6(0, 2, 0, 1, 1, 0) << 12;
constexpr unsigned kOffY = pack6(0, 0, 2, 0, 1, 1) | pack6(0, 2, 2, 1, 2, 1) << 12;
__device__ __forceinline__ int off_x(int t, int b) { return (int)(kOffX >> (12 * t + 2 * b)) & 3; }
__device__ __forceinline__ int off_y(int t, int b) { return (int)(kOffY >> (12 * t + 2 * b)) & 3; }

// One row: returns false (and does nothing) when the window exceeds CAP nodes.  The block is
// one wavefront; every thread takes the same path.  The window is in LDS (CAP > 0), or, with
// CAP = 0, in device memory at gflag / gval (room for the row's window; each window position
// is written by one lane only after the marking pass, so the sums keep their fixed order).
// Rows whose window exceeds kWinCap (the wide form) are listed in huge = [count, largest
// window, rows...] for the device-memory form.
// Adjacency entries [qa, min(qa + 64, q1)) of a row, one per lane: the entry (element << 2 |
// local node) and its element's piece range.  Returns the number of entries.
__device__ __forceinline__ int load_adj(int qa, int q1, const int *__restrict__ n2e,
                                        const int *__restrict__ e_piece, int &av, int &aps, int &ape) {
  const int lane = threadIdx.x;
  const int A = min(kWave, q1 - qa);
  av = 0;
  aps = ape = 0;
  if (lane < A) {
    av = n2e[qa + lane];
    aps = e_piece[av >> 2];
    ape = e_piece[(av >> 2) + 1];
  }
  return A;
}

template <int CAP>
__device__ bool cf_row(int64_t l, int pass, int n, const int *__restrict__ n2e_ptr, const int *__restrict__ n2e,
                       const int *__restrict__ e_piece, const int *__restrict__ pair_T,
                       const double *__restrict__ piece_L, int *cnt, const int *rowptr, int *col, double *val,
                       int *flag, int *huge = nullptr, int *gflag = nullptr, double *gval = nullptr) {
  constexpr int SCAP = CAP > 0 ? CAP : 1;
  // windows of up to kWinSmall nodes keep their sums in registers (NACC per lane)
  constexpr int NACC = CAP > 0 && CAP <= 256 ? CAP / kWave : 1;
  __shared__ int sflag[SCAP];
  __shared__ double sval[NACC > 1 ? 1 : SCAP];
  __shared__ int kslot[kWave], kT[kWave];
  int *wflag = CAP > 0 ? sflag : gflag;
  double *wval = CAP > 0 ? sval : gval;
  int lane = threadIdx.x;
  const int L = 2 * n + 1;
  // window of lattice nodes covered by the pieces around node l.  The adjacency entries are
  // read a wavefront at a time (lane i: entry qa + i, its element's first and end piece) and
  // passed to every lane by shuffles.
  int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
  const int q0 = n2e_ptr[l], q1 = n2e_ptr[l + 1];
  int av, aps, ape;
  for (int qa = q0; qa < q1; qa += kWave) {
    const int A = load_adj(qa, q1, n2e, e_piece, av, aps, ape);
    for (int i = 0; i < A; ++i) {
      const int ps = __shfl(aps, i, kWave), pe = __shfl(ape, i, kWave);
      for (int p = ps + lane; p < pe; p += kWave) {
        int T = pair_T[p];
        if (T < 0) continue;   // an empty slot of the time-coherent layout
        int cell = T >> 1;
        int ci = cell % n, cj = cell / n;
        imin = min(imin, 2 * ci); imax = max(imax, 2 * ci + 2);
        jmin = min(jmin, 2 * cj); jmax = max(jmax, 2 * cj + 2);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    imin = min(imin, __shfl_xor(imin, off, kWave));
    imax = max(imax, __shfl_xor(imax, off, kWave));
    jmin = min(jmin, __shfl_xor(jmin, off, kWave));
    jmax = max(jmax, __shfl_xor(jmax, off, kWave));
  }
  if (imax < 0) {              // no pieces (cannot happen for a valid map)
    if (!pass && lane == 0) cnt[l] = 0;
    return true;
  }
  int wI = imax - imin + 1, wJ = jmax - jmin + 1;
  int W = wI * wJ;
  if (CAP > 0 && W > CAP) {
    if (CAP < kWinCap) return false;   // left to the wide form
    if (!pass && lane == 0) {          // left to the device-memory form (listed once)
      huge[2 + atomicAdd(&huge[0], 1)] = (int)l;
      atomicMax(&huge[1], W);
    }
    return true;
  }
  for (int p = lane; p < W; p += kWave) {
    wflag[p] = 0;
    if (NACC == 1) wval[p] = 0.0;
  }
  __syncthreads();
  // mark the columns
  for (int qa = q0; qa < q1; qa += kWave) {
    const int A = load_adj(qa, q1, n2e, e_piece, av, aps, ape);
    for (int i = 0; i < A; ++i) {
      const int ps = __shfl(aps, i, kWave), pe = __shfl(ape, i, kWave);
      for (int p = ps + lane; p < pe; p += kWave) {
        int T = pair_T[p], t = T & 1, cell = T >> 1;
        if (T < 0) continue;
        int ci = cell % n, cj = cell / n;
        for (int b = 0; b < 6; ++b) {
          int I = 2 * ci + off_x(t, b) - imin, J = 2 * cj + off_y(t, b) - jmin;
          wflag[J * wI + I] = 1;
        }
      }
    }
  }
  __syncthreads();
  if (!pass) {
    int c = 0;
    for (int p = lane; p < W; p += kWave) c += wflag[p];
    c = wave_sum(c);
    if (lane == 0) cnt[l] = c;
    return true;
  }
  // values: item order is fixed (adjacency, piece, local node); window position p is summed
  // by lane p % 64 only, so the order of every sum is fixed.  For each element, 64 slots at a
  // time: the kept ones are listed in slot order (ballot), then the items of up to 10 kept
  // pieces (lane 6 k + b: piece k, local node b) find their window positions and values at once,
  // and every lane walks them in item order, adding those it owns (in registers for the small
  // windows, in the window array otherwise).
  double acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
  for (int qa = q0; qa < q1; qa += kWave) {
    const int A = load_adj(qa, q1, n2e, e_piece, av, aps, ape);
    for (int i = 0; i < A; ++i) {
      const int a = __shfl(av, i, kWave) & 3;
      const int ps = __shfl(aps, i, kWave), pe = __shfl(ape, i, kWave);
      for (int sb = ps; sb < pe; sb += kWave) {
        const int sl = sb + lane;
        const int Tl = sl < pe ? pair_T[sl] : -1;
        const uint64_t kept = __ballot(Tl >= 0);
        const int nk = __popcll(kept);
        if (Tl >= 0) {
          const int r = __popcll(kept & ((1ull << lane) - 1));
          kslot[r] = sl;
          kT[r] = Tl;
        }
        __syncthreads();
        for (int k0 = 0; k0 < nk; k0 += 10) {
          const int m = 6 * min(10, nk - k0);
          int posl = -1;
          double vl = 0.0;
          if (lane < m) {
            const int k = k0 + lane / 6, b = lane % 6;
            const int T = kT[k], t = T & 1, cell = T >> 1;
            const int ci = cell % n, cj = cell / n;
            posl = (2 * cj + off_y(t, b) - jmin) * wI + 2 * ci + off_x(t, b) - imin;
            vl = piece_L[18 * (int64_t)kslot[k] + a * 6 + b];
          }
          // item it is read from lane it (uniform position, so the sum it belongs to is chosen
          // by a scalar branch; only the owning lane adds)
          for (int it = 0; it < m; ++it) {
            const int pos = __builtin_amdgcn_readlane(posl, it);
            const double v = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(vl), it),
                                              __builtin_amdgcn_readlane(__double2loint(vl), it));
            const bool own = (pos & (kWave - 1)) == lane;
            if (NACC > 1) {
              const int k = pos >> 6;
#pragma unroll
              for (int kk = 0; kk < NACC; ++kk)
                if (k == kk) acc[kk] = own ? acc[kk] + v : acc[kk];
            } else if (own) {
              wval[pos] += v;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // compact in window order (= ascending column index)
  int base = rowptr[l];
  for (int p0 = 0; p0 < W; p0 += kWave) {
    int p = p0 + lane;
    int f = (p < W) ? wflag[p] : 0;
    int incl = f;
    for (int off = 1; off < kWave; off <<= 1) {
      int t = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += t;
    }
    if (f) {
      int I = imin + p % wI, J = jmin + p / wI;
      bool bndc = I == 0 || J == 0 || I == 2 * n || J == 2 * n;
      col[base + incl - 1] = J * L + I;
      double v = 0.0;
      if (NACC > 1) {
#pragma unroll
        for (int k = 0; k < NACC; ++k)
          if (k == p0 / kWave) v = acc[k];
      } else {
        v = wval[p];
      }
      val[base + incl - 1] = bndc ? 0.0 : v;
    }
    base += __shfl(incl, kWave - 1, kWave);
  }
  return true;
}


// Rows with a window of up to kWinSmall nodes (3 KB of LDS: many wavefronts per CU; the
// windows of a solid about as fine as the fluid grid span a few cells); the others are listed
// (defer[0] = count) for the wider forms below.
constexpr int kWinSmall = 256;
constexpr int kWinMid = 1024;
__global__ void __launch_bounds__(kWave) k_cf_rows(int pass, int64_t ns, int n, const int *__restrict__ n2e_ptr,
                                                   const int *__restrict__ n2e, const int *__restrict__ e_piece,
                                                   const int *__restrict__ pair_T,
                                                   const double *__restrict__ piece_L, int *cnt, const int *rowptr,
                                                   int *col, double *val, int *flag, int *defer) {
  const int64_t l = blockIdx.x;
  if (l >= ns) return;
  if (!cf_row<kWinSmall>(l, pass, n, n2e_ptr, n2e, e_piece, pair_T, piece_L, cnt, rowptr, col, val, flag) &&
      threadIdx.x == 0)
    defer[1 + atomicAdd(&defer[0], 1)] = (int)l;   // list order does not matter: rows are independent
}

// The rows listed in `in` with a window of up to CAP nodes (grid-stride over the list); rows
// with larger windows go to the list `out` (CAP < kWinCap) or to huge (CAP = kWinCap).
template <int CAP>
__global__ void __launch_bounds__(kWave) k_cf_rows_wide(int pass, int n, const int *__restrict__ n2e_ptr,
                                                        const int *__restrict__ n2e, const int *__restrict__ e_piece,
                                                        const int *__restrict__ pair_T,
                                                        const double *__restrict__ piece_L, int *cnt,
                                                        const int *rowptr, int *col, double *val, int *flag,
                                                        const int *in, int *out, int *huge) {
  const int count = in[0];
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int l = in[1 + q];
    if (!cf_row<CAP>(l, pass, n, n2e_ptr, n2e, e_piece, pair_T, piece_L, cnt, rowptr, col, val, flag, huge) &&
        threadIdx.x == 0)
      out[1 + atomicAdd(&out[0], 1)] = l;
    __syncthreads();
  }
}

// The three LDS forms of one pass over all rows: small windows (one wavefront per row), then
// the listed rows of up to kWinMid and kWinCap nodes; rows above that are listed in huge.
static void cf_rows_lds(hipStream_t s, int pass, int64_t ns, int n, const int *n2e_ptr, const int *n2e,
                        const int *e_piece, const int *pair_T, const double *piece_L, int *cnt, const int *rowptr,
                        int *col, double *val, int *flag, int *defer, int *defer2, int *huge) {
  fill(defer, 1, 0, s);
  fill(defer2, 1, 0, s);
  hipLaunchKernelGGL(k_cf_rows, dim3((unsigned)ns), dim3(kWave), 0, s, pass, ns, n, n2e_ptr, n2e, e_piece, pair_T,
                     piece_L, cnt, rowptr, col, val, flag, defer);
  hipLaunchKernelGGL(k_cf_rows_wide<kWinMid>, dim3(1024), dim3(kWave), 0, s, pass, n, n2e_ptr, n2e, e_piece, pair_T,
                     piece_L, cnt, rowptr, col, val, flag, defer, defer2, huge);
  hipLaunchKernelGGL(k_cf_rows_wide<kWinCap>, dim3(256), dim3(kWave), 0, s, pass, n, n2e_ptr, n2e, e_piece, pair_T,
                     piece_L, cnt, rowptr, col, val, flag, defer2, nullptr, huge);
  FSI_CHECK_LAUNCH();
}

// The rows with windows above kWinCap nodes (a solid much coarser than the fluid grid), one
// after another on one wavefront, each with its window in device memory (flags, values: the
// largest window listed, huge[1] entries each).
__global__ void __launch_bounds__(kWave) k_cf_rows_huge(int pass, int n, const int *__restrict__ n2e_ptr,
                                                        const int *__restrict__ n2e, const int *__restrict__ e_piece,
                                                        const int *__restrict__ pair_T,
                                                        const double *__restrict__ piece_L, int *cnt,
                                                        const int *rowptr, int *col, double *val, int *flag,
                                                        const int *huge, int *gflag, double *gval) {
  const int count = huge[0];
  for (int q = 0; q < count; ++q) {
    cf_row<0>(huge[2 + q], pass, n, n2e_ptr, n2e, e_piece, pair_T, piece_L, cnt, rowptr, col, val, flag, nullptr,
              gflag, gval);
    __syncthreads();
  }
}

// ---- transpose
__global__ void k_count_cols(int64_t nnz, const int *col, int *cnt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_scatter_t(int64_t nrows, const int *rowptr, const int *col, const double *val,
                            const int *tptr, int *fill, int *tcol, double *tval, int *tsrc) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    int c = col[k];
    int pos = tptr[c] + atomicAdd(&fill[c], 1);
    tcol[pos] = (int)r;
    tval[pos] = val[k];
    if (tsrc) tsrc[pos] = k;
  }
}

// Ordering of the transposed rows.  The scatter above places the entries of a row of
// C_f^T in an arbitrary order (atomic slots); each entry is then moved to its rank among the
// solid-node indices of its row (unique within a row), so the result is deterministic.
// Rows of up to kShortRow entries are ranked by one thread; longer rows (a solid much finer
// than the fluid grid puts thousands of solid nodes in one P2 support) are listed and ranked
// by a workgroup each, with the row's keys staged through LDS in chunks.
constexpr int kShortRow = 32;
constexpr int kRankChunk = 4096;

__global__ void k_rank_short(int64_t nrows, const int *rowptr, const int *tcol, const double *tval, int *col,
                             double *val, int *long_rows, const int *tsrc, int *perm) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int k0 = rowptr[r], k1 = rowptr[r + 1];
  if (k1 - k0 > kShortRow) {
    long_rows[1 + atomicAdd(&long_rows[0], 1)] = (int)r;   // list order does not matter
    return;
  }
  for (int i = k0; i < k1; ++i) {
    const int c = tcol[i];
    int rank = 0;
    for (int j = k0; j < k1; ++j) rank += tcol[j] < c;
    col[k0 + rank] = c;
    val[k0 + rank] = tval[i];
    if (perm) perm[k0 + rank] = tsrc[i];
  }
}

// One workgroup per listed row (grid-stride over the list; the count is read on the device).
__global__ void __launch_bounds__(256) k_rank_long(const int *rowptr, const int *tcol, const double *tval, int *col,
                                                   double *val, const int *long_rows, const int *tsrc, int *perm) {
  __shared__ int keys[kRankChunk];
  const int count = long_rows[0];
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int r = long_rows[1 + q];
    const int k0 = rowptr[r], k1 = rowptr[r + 1], len = k1 - k0;
    // this thread's elements: i = k0 + threadIdx.x + 256 t (at most kRankMine per pass)
    for (int base = 0; base < len; base += 256 * 8) {
      int mine[8], rank[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = base + threadIdx.x + 256 * t;
        mine[t] = i < len ? tcol[k0 + i] : 0;
        rank[t] = 0;
      }
      for (int c0 = 0; c0 < len; c0 += kRankChunk) {
        const int cl = min(kRankChunk, len - c0);
        __syncthreads();
        for (int j = threadIdx.x; j < cl; j += 256) keys[j] = tcol[k0 + c0 + j];
        __syncthreads();
        for (int j = 0; j < cl; ++j) {
          const int kj = keys[j];   // same address for the whole workgroup: broadcast
#pragma unroll
          for (int t = 0; t < 8; ++t) rank[t] += kj < mine[t];
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = base + threadIdx.x + 256 * t;
        if (i < len) {
          col[k0 + rank[t]] = mine[t];
          val[k0 + rank[t]] = tval[k0 + i];
          if (perm) perm[k0 + rank[t]] = tsrc[k0 + i];
        }
      }
    }
    __syncthreads();
  }
}

static int read_int(const int *d, hipStream_t s) {
  int h = 0;
  FSI_HIP(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  return h;
}

static void check_flags(int *flag, hipStream_t s) {
  int f = read_int(flag, s);
  if (f) fill(flag, 1, 0, s);
  FSI_REQUIRE(!(f & DF_MESH), FSI_E_MESH, "X^n maps a solid triangle to a degenerate/inverted triangle or outside [0,1]^2");
}

// Where one assembly keeps its work arrays and finds its outputs.
//  GrowWork: the context's grow-only buffers (fsi_assemble_coupling).
//  ArenaWork: consecutive 256-byte aligned pieces of the per-device static array below
//  (fsi_assemble_coupling_noalloc); the outputs must fit the context's coupling storage.
struct GrowWork {
  Ctx &c;
  int *flags() {
    if (!c.dflag.p) {
      c.dflag.alloc(4);
      fill(c.dflag.p, 4, 0, c.stream);
    }
    return c.dflag.p;
  }
  template <typename T>
  T *work(DevBuf<T> &b, int64_t n, const char *) {
    b.reserve((size_t)n);
    return b.p;
  }
  int *scan(int64_t n) {
    c.scan_tmp.reserve((size_t)scan_tmp_len(n));
    return c.scan_tmp.p;
  }
  template <typename T>
  T *out(DevBuf<T> &b, int64_t n, const char *) {
    b.reserve((size_t)n);
    return b.p;
  }
};

struct ArenaWork {
  Ctx &c;
  unsigned char *base;
  size_t cap, used;
  template <typename T>
  T *carve(int64_t n, const char *what) {
    const size_t bytes = (((size_t)(n > 0 ? n : 1) * sizeof(T)) + 255) & ~(size_t)255;
    FSI_REQUIRE(used + bytes <= cap, FSI_E_CAPACITY,
                std::string("allocation-free coupling assembly: the work space (") + what + " and before it: " +
                    std::to_string(used + bytes) + " bytes) exceeds the " + std::to_string(cap >> 20) +
                    " MiB scratch array; use fsi_assemble_coupling");
    T *p = (T *)(base + used);
    used += bytes;
    return p;
  }
  int *flags() {
    int *f = carve<int>(4, "error flags");
    fill(f, 4, 0, c.stream);   // the array keeps the previous call's contents
    return f;
  }
  template <typename T>
  T *work(DevBuf<T> &, int64_t n, const char *what) { return carve<T>(n, what); }
  int *scan(int64_t n) { return carve<int>(scan_tmp_len(n), "scan partials"); }
  template <typename T>
  T *out(DevBuf<T> &b, int64_t n, const char *what) {
    FSI_REQUIRE(b.p && (int64_t)b.n >= n, FSI_E_CAPACITY,
                std::string("allocation-free coupling assembly: ") + what + " needs " + std::to_string(n) +
                    " entries, the context's coupling storage holds " + std::to_string(b.p ? b.n : 0) +
                    "; fsi_assemble_coupling grows it");
    return b.p;
  }
};

template <typename Work>
static void build_transpose(Ctx &c, Work &w, int nnz, bool keep_perm);

// Rows of C_f from a piece list (e_piece: the first slot of each element; empty slots have
// pair_T < 0), then C_f^T and the FP32 copies.  perm, when given, receives for every C_f^T
// entry the index of its C_f entry (the time-coherent form refills C_f^T values with it).
template <typename Work>
static void build_rows(Ctx &c, Work &w, const int *e_piece, const int *pair_T, const double *piece_L, int *flag,
                       bool keep_perm) {
  hipStream_t s = c.stream;
  const int64_t ns = c.Ns;
  const int n = c.n;
  Csr &Cf = c.Cf;
  Cf.nrows = ns;
  Cf.ncols = c.N2;
  Cf.width = 1;
  int *cf_rp = w.out(Cf.rowptr, ns + 1, "the C_f row pointers");
  int *defer = w.work(c.cf_defer, ns + 1, "deferred rows");
  int *defer2 = w.work(c.cf_defer2, ns + 1, "deferred rows");
  int *huge = w.work(c.cf_huge, ns + 2, "rows with large windows");
  fill(huge, 2, 0, s);
  cf_rows_lds(s, 0, ns, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T, piece_L, cf_rp, nullptr, nullptr, nullptr, flag,
              defer, defer2, huge);
  // rows whose window exceeds the LDS form: a device-memory window of the largest size
  int hcnt[2] = {0, 0};
  FSI_HIP(hipMemcpyAsync(hcnt, huge, sizeof(hcnt), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  c.cf_hcnt[0] = hcnt[0];
  c.cf_hcnt[1] = hcnt[1];
  int *gflag = nullptr;
  double *gval = nullptr;
  if (hcnt[0] > 0) {
    gflag = w.work(c.cf_wflag, hcnt[1], "the large window");
    gval = w.work(c.cf_wval, hcnt[1], "the large window");
    hipLaunchKernelGGL(k_cf_rows_huge, dim3(1), dim3(kWave), 0, s, 0, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T,
                       piece_L, cf_rp, nullptr, nullptr, nullptr, flag, huge, gflag, gval);
    FSI_CHECK_LAUNCH();
  }
  scan_excl(cf_rp, cf_rp, ns, w.scan(ns), s);
  check_flags(flag, s);
  const int nnz = read_int(cf_rp + ns, s);
  Cf.nnz = nnz;
  int *cf_col = w.out(Cf.col, nnz, "C_f");
  double *cf_val = w.out(Cf.val, nnz, "C_f");
  cf_rows_lds(s, 1, ns, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T, piece_L, nullptr, cf_rp, cf_col, cf_val, flag,
              defer, defer2, huge);
  if (hcnt[0] > 0)
    hipLaunchKernelGGL(k_cf_rows_huge, dim3(1), dim3(kWave), 0, s, 1, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T,
                       piece_L, nullptr, cf_rp, cf_col, cf_val, flag, huge, gflag, gval);
  FSI_CHECK_LAUNCH();
  build_transpose(c, w, nnz, keep_perm);
}

// C_f^T of the rows in c.Cf (nnz entries) and the FP32 copies of both; perm as for build_rows.
template <typename Work>
static void build_transpose(Ctx &c, Work &w, int nnz, bool keep_perm) {
  hipStream_t s = c.stream;
  const int64_t ns = c.Ns;
  const int *cf_rp = c.Cf.rowptr.p, *cf_col = c.Cf.col.p;
  const double *cf_val = c.Cf.val.p;
  // C_f^T
  Csr &Ct = c.CfT;
  Ct.nrows = c.N2;
  Ct.ncols = ns;
  Ct.width = 1;
  Ct.nnz = nnz;
  int *ct_rp = w.out(Ct.rowptr, c.N2 + 1, "the C_f^T row pointers");
  int *ct_fill = w.work(c.cft_fill, c.N2, "transpose fill counters");
  fill(ct_rp, c.N2 + 1, 0, s);
  fill(ct_fill, c.N2, 0, s);
  hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256)), dim3(256), 0, s, (int64_t)nnz, cf_col, ct_rp);
  scan_excl(ct_rp, ct_rp, c.N2, w.scan(c.N2), s);
  int *ct_col = w.out(Ct.col, nnz, "C_f^T");
  double *ct_val = w.out(Ct.val, nnz, "C_f^T");
  int *tcol = w.work(c.cft_tcol, nnz, "transpose staging");
  double *tval = w.work(c.cft_tval, nnz, "transpose staging");
  int *tsrc = keep_perm ? w.work(c.cft_tsrc, nnz, "transpose staging") : nullptr;
  int *perm = keep_perm ? w.work(c.cft_perm, nnz, "transpose permutation") : nullptr;
  int *long_rows = w.work(c.cft_long, c.N2 + 1, "long transposed rows");
  fill(long_rows, 1, 0, s);
  hipLaunchKernelGGL(k_scatter_t, dim3(grid_for(ns, 256)), dim3(256), 0, s, ns, cf_rp, cf_col, cf_val, ct_rp,
                     ct_fill, tcol, tval, tsrc);
  hipLaunchKernelGGL(k_rank_short, dim3(grid_for(c.N2, 256)), dim3(256), 0, s, c.N2, ct_rp, tcol, tval, ct_col,
                     ct_val, long_rows, tsrc, perm);
  hipLaunchKernelGGL(k_rank_long, dim3(512), dim3(256), 0, s, ct_rp, tcol, tval, ct_col, ct_val, long_rows, tsrc,
                     perm);
  FSI_CHECK_LAUNCH();
  float *cf32 = w.out(c.Cf.val32, nnz, "the FP32 copy of C_f");
  float *ct32 = w.out(Ct.val32, nnz, "the FP32 copy of C_f^T");
  convert(cf32, cf_val, nnz, s);
  convert(ct32, ct_val, nnz, s);
  c.have_cf = true;
}

template <typename Work>
static void assemble(Ctx &c, const double *Xn, Work &w) {
  hipStream_t s = c.stream;
  const int64_t nt = c.Nt, ns = c.Ns;
  const int n = c.n;
  c.have_cf = false;
  c.pairs_kept = false;
  c.inc_valid = false;   // the piece list below replaces the time-coherent slots
  int *flag = w.flags();
  int *cand_off = w.work(c.cand_off, nt + 1, "candidate offsets");
  hipLaunchKernelGGL(k_cand_count, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, ns, n, Xn, c.tri.p, cand_off,
                     flag);
  FSI_CHECK_LAUNCH();
  scan_excl(cand_off, cand_off, nt, w.scan(nt), s);
  check_flags(flag, s);
  const int ncand = read_int(cand_off + nt, s);
  c.n_cand = ncand;
  int *piece_off = w.work(c.piece_cnt, (int64_t)ncand + 1, "piece counters");
  hipLaunchKernelGGL(k_clip_count, dim3(grid_for(ncand, 128)), dim3(128), 0, s, (int64_t)ncand, nt, ns, n, Xn,
                     c.tri.p, cand_off, piece_off);
  FSI_CHECK_LAUNCH();
  scan_excl(piece_off, piece_off, ncand, w.scan(ncand), s);
  const int npieces = read_int(piece_off + ncand, s);
  c.n_pairs = npieces;
  int *pair_E = w.work(c.pair_E, npieces, "piece list");
  int *pair_T = w.work(c.pair_T, npieces, "piece list");
  double *piece_L = w.work(c.piece_L, 18 * (int64_t)npieces, "piece matrices");
  hipLaunchKernelGGL(k_clip_emit, dim3(grid_for(ncand, 128)), dim3(128), 0, s, (int64_t)ncand, nt, ns, n, Xn,
                     c.tri.p, c.ref_area.p, cand_off, piece_off, pair_E, pair_T, piece_L);
  int *e_piece = w.work(c.e_piece, nt + 1, "element piece offsets");
  hipLaunchKernelGGL(k_elem_piece_off, dim3(grid_for(nt + 1, 256)), dim3(256), 0, s, nt, cand_off, piece_off,
                     e_piece);
  FSI_CHECK_LAUNCH();
  build_rows(c, w, e_piece, pair_T, piece_L, flag, false);
}

// ---- the time-coherent form (Sec. 7: follow the solid from its position at the previous
// step instead of detecting its intersections anew)
//
// A rebuild gives every element a candidate box of (w + 1) x (h + 1) cells, one more than its
// bounding box spans in each direction, and two piece slots per candidate cell (the fluid
// triangles T0, T1 of the cell; pair_T = -1 for an empty slot).  A later call re-clips only
// the elements whose vertices moved (any coordinate differs from the previous call's), into
// the same slots: the candidate q of an element is cell (i0 + q mod w, j0 + q div w) of its
// current box, as in the full assembly, so the kept pieces come in the same order and every
// C_f sum in the same order (the result is bitwise that of the full assembly).  Then
//   - nothing moved: C_f and C_f^T are kept;
//   - some moved element's kept pieces (read in slot order) differ from its previous ones:
//     rows, pattern and transpose anew;
//   - otherwise the piece list, and so the pattern, is kept: row values again (pass 1 of the
//     rows) and C_f^T values through the stored permutation;
//   - an element outgrew its box: a rebuild.
enum { IF_MESH = 1, IF_OVERFLOW = 2, IF_PATTERN = 4 };

// Rebuild: validity and the candidate box of every element.
__global__ void k_inc_box(int64_t nt, int64_t ns, int n, const double *__restrict__ X, const int *__restrict__ tri,
                          int *box, int *cnt, int *moved, int *flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  Pt P[3];
  load_tri(X, ns, tri, (int)e, P);
  bool ok = tri_area(P) > 0.0;
  for (int m = 0; m < 3; ++m)
    ok = ok && P[m].x >= 0.0 && P[m].x <= 1.0 && P[m].y >= 0.0 && P[m].y <= 1.0;
  moved[e] = 1;
  if (!ok) {
    atomicOr(flag, IF_MESH);
    box[2 * e] = box[2 * e + 1] = 0;
    cnt[e] = 0;
    return;
  }
  int i0, i1, j0, j1;
  cell_range(P, n, i0, i1, j0, j1);
  const int cw = min(i1 - i0 + 2, n), ch = min(j1 - j0 + 2, n);
  box[2 * e] = cw;
  box[2 * e + 1] = ch;
  cnt[e] = cw * ch;
}

// A later call: validity, which elements moved, and whether one outgrew its box.
// inc[0]: flags, inc[1]: moved elements.
__global__ void k_inc_moved(int64_t nt, int64_t ns, int n, const double *__restrict__ X,
                            const double *__restrict__ Xold, const int *__restrict__ tri, const int *__restrict__ box,
                            int *moved, int *inc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  Pt P[3];
  load_tri(X, ns, tri, (int)e, P);
  bool mv = false;
  for (int m = 0; m < 3; ++m) {
    const int v = tri[3 * e + m];
    mv = mv || P[m].x != Xold[v] || P[m].y != Xold[ns + v];
  }
  moved[e] = mv ? 1 : 0;
  if (!mv) return;   // unchanged since a call that found it valid
  atomicAdd(&inc[1], 1);
  bool ok = tri_area(P) > 0.0;
  for (int m = 0; m < 3; ++m)
    ok = ok && P[m].x >= 0.0 && P[m].x <= 1.0 && P[m].y >= 0.0 && P[m].y <= 1.0;
  if (!ok) {
    atomicOr(&inc[0], IF_MESH);
    return;
  }
  int i0, i1, j0, j1;
  cell_range(P, n, i0, i1, j0, j1);
  if (i1 - i0 + 1 > box[2 * e] || j1 - j0 + 1 > box[2 * e + 1]) atomicOr(&inc[0], IF_OVERFLOW);
}

// Re-clip the candidate slots of the moved elements; the previous piece of each slot goes to
// prevT.  inc[2] keeps the number of kept pieces.  An element that outgrew its box (the host
// then rebuilds) or is invalid (the call fails) only writes within its own slots.
__global__ void k_inc_emit(int64_t nslot, int64_t nt, int64_t ns, int n, const double *__restrict__ X,
                           const int *__restrict__ tri, const double *__restrict__ ref_area,
                           const int *__restrict__ cand_off, const int *__restrict__ moved, int *pair_E, int *pair_T,
                           int *prevT, double *piece_L, int *inc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nslot) return;
  const int e = find_owner(cand_off, nt, c);
  if (!moved[e]) return;
  Pt P[3];
  load_tri(X, ns, tri, e, P);
  int i0, i1, j0, j1;
  cell_range(P, n, i0, i1, j0, j1);
  const int w = i1 - i0 + 1;
  const int q = (int)(c - cand_off[e]);
  Pt qq[2][kMaxPoly];
  int mq[2] = {0, 0};
  int mask = 0, i = 0, j = 0;
  const double area = tri_area(P);
  if (area > 0.0 && q < w * (j1 - j0 + 1)) {
    i = i0 + q % w;
    j = j0 + q / w;
    mask = clip_pieces(P, n, i, j, qq, mq);
  }
  int delta = 0;
  for (int t = 0; t < 2; ++t) {
    const int64_t sl = 2 * c + t;
    const int Tn = (mask >> t) & 1 ? 2 * (j * n + i) + t : -1;
    const int To = pair_T[sl];
    delta += (Tn >= 0) - (To >= 0);
    prevT[sl] = To;
    pair_T[sl] = Tn;
    pair_E[sl] = Tn >= 0 ? e : -1;
    if (Tn >= 0) piece_matrix(P, qq[t], mq[t], i, j, t, n, ref_area[e] / area, piece_L + 18 * sl);
  }
  if (delta) atomicAdd(&inc[2], delta);
}

// inc[0] |= IF_PATTERN when a moved element's kept pieces, read in slot order, differ from
// its previous ones.  A box that shifted with the same pieces keeps the piece list (and so
// every row of C_f, with its sums in the same order).
__global__ void k_inc_cmp(int64_t nt, const int *__restrict__ cand_off, const int *__restrict__ moved,
                          const int *__restrict__ pair_T, const int *__restrict__ prevT, int *inc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt || !moved[e]) return;
  const int64_t s1 = 2 * (int64_t)cand_off[e + 1];
  int64_t a = 2 * (int64_t)cand_off[e], b = a;
  for (;;) {
    while (a < s1 && pair_T[a] < 0) ++a;
    while (b < s1 && prevT[b] < 0) ++b;
    if (a == s1 || b == s1) {
      if (a != s1 || b != s1) atomicOr(&inc[0], IF_PATTERN);
      return;
    }
    if (pair_T[a] != prevT[b]) {
      atomicOr(&inc[0], IF_PATTERN);
      return;
    }
    ++a;
    ++b;
  }
}

__global__ void k_inc_slot_off(int64_t nt, const int *cand_off, int *e_piece) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e <= nt) e_piece[e] = 2 * cand_off[e];
}

__global__ void k_gather_vals(int64_t nnz, const int *__restrict__ perm, const double *__restrict__ src,
                              double *__restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) dst[k] = src[perm[k]];
}

// Pattern kept: C_f values by pass 1 of the rows (row pointers, deferred and large-window
// lists as built), C_f^T values through the permutation.
static void refill_values(Ctx &c) {
  hipStream_t s = c.stream;
  const int64_t ns = c.Ns, nnz = c.Cf.nnz;
  const int n = c.n;
  const int *e_piece = c.e_piece.p, *pair_T = c.pair_T.p;
  const double *piece_L = c.piece_L.p;
  cf_rows_lds(s, 1, ns, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T, piece_L, nullptr, c.Cf.rowptr.p, c.Cf.col.p,
              c.Cf.val.p, nullptr, c.cf_defer.p, c.cf_defer2.p, c.cf_huge.p);
  if (c.cf_hcnt[0] > 0)
    hipLaunchKernelGGL(k_cf_rows_huge, dim3(1), dim3(kWave), 0, s, 1, n, c.n2e_ptr.p, c.n2e.p, e_piece, pair_T,
                       piece_L, nullptr, c.Cf.rowptr.p, c.Cf.col.p, c.Cf.val.p, nullptr, c.cf_huge.p, c.cf_wflag.p,
                       c.cf_wval.p);
  hipLaunchKernelGGL(k_gather_vals, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, c.cft_perm.p, c.Cf.val.p,
                     c.CfT.val.p);
  FSI_CHECK_LAUNCH();
  convert(c.Cf.val32.p, c.Cf.val.p, nnz, s);
  convert(c.CfT.val32.p, c.CfT.val.p, nnz, s);
}

static void assemble_incremental(Ctx &c, const double *Xn) {
  hipStream_t s = c.stream;
  const int64_t nt = c.Nt, ns = c.Ns;
  const int n = c.n;
  GrowWork w{c};
  ++c.inc_counts[0];
  if (!c.inc_flag.p) c.inc_flag.alloc(4);
  int *inc = c.inc_flag.p;
  if (c.inc_valid && c.have_cf) {
    fill(inc, 2, 0, s);
    hipLaunchKernelGGL(k_inc_moved, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, ns, n, Xn, c.inc_X.p, c.tri.p,
                       c.inc_box.p, c.inc_moved.p, inc);
    hipLaunchKernelGGL(k_inc_emit, dim3(grid_for(c.n_cand, 128)), dim3(128), 0, s, c.n_cand, nt, ns, n, Xn,
                       c.tri.p, c.ref_area.p, c.cand_off.p, c.inc_moved.p, c.pair_E.p, c.pair_T.p, c.inc_prevT.p,
                       c.piece_L.p, inc);
    hipLaunchKernelGGL(k_inc_cmp, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, c.cand_off.p, c.inc_moved.p,
                       c.pair_T.p, c.inc_prevT.p, inc);
    FSI_CHECK_LAUNCH();
    FSI_HIP(hipMemcpyAsync(c.inc_X.p, Xn, 2 * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
    int h[3] = {0, 0, 0};
    FSI_HIP(hipMemcpyAsync(h, inc, sizeof(h), hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    if (h[0] & IF_MESH) {
      c.inc_valid = false;
      c.have_cf = false;
      FSI_REQUIRE(false, FSI_E_MESH, "X^n maps a solid triangle to a degenerate/inverted triangle or outside [0,1]^2");
    }
    if (!(h[0] & IF_OVERFLOW)) {
      c.n_pairs = h[2];
      if (h[1] == 0) {
        ++c.inc_counts[4];          // nothing moved: C_f as it is
      } else if (!(h[0] & IF_PATTERN)) {
        refill_values(c);
        ++c.inc_counts[3];
      } else {
        c.have_cf = false;
        build_rows(c, w, c.e_piece.p, c.pair_T.p, c.piece_L.p, w.flags(), true);
        ++c.inc_counts[2];
      }
      return;
    }
  }
  // rebuild: boxes, slots, every element clipped
  ++c.inc_counts[1];
  c.inc_valid = false;
  c.have_cf = false;
  c.pairs_kept = false;
  int *box = w.work(c.inc_box, 2 * nt, "candidate boxes");
  int *moved = w.work(c.inc_moved, nt, "moved flags");
  double *xold = w.work(c.inc_X, 2 * ns, "previous positions");
  int *cand_off = w.work(c.cand_off, nt + 1, "candidate offsets");
  fill(inc, 4, 0, s);
  hipLaunchKernelGGL(k_inc_box, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, ns, n, Xn, c.tri.p, box, cand_off,
                     moved, inc);
  FSI_CHECK_LAUNCH();
  scan_excl(cand_off, cand_off, nt, w.scan(nt), s);
  int h[2] = {0, 0};
  FSI_HIP(hipMemcpyAsync(&h[0], inc, sizeof(int), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipMemcpyAsync(&h[1], cand_off + nt, sizeof(int), hipMemcpyDeviceToHost, s));
  FSI_HIP(hipStreamSynchronize(s));
  FSI_REQUIRE(!(h[0] & IF_MESH), FSI_E_MESH,
              "X^n maps a solid triangle to a degenerate/inverted triangle or outside [0,1]^2");
  const int64_t nslot = h[1];
  c.n_cand = nslot;
  int *pair_E = w.work(c.pair_E, 2 * nslot, "piece slots");
  int *pair_T = w.work(c.pair_T, 2 * nslot, "piece slots");
  int *prevT = w.work(c.inc_prevT, 2 * nslot, "previous piece slots");
  double *piece_L = w.work(c.piece_L, 36 * nslot, "piece matrices");
  int *e_piece = w.work(c.e_piece, nt + 1, "element slot offsets");
  fill(pair_T, 2 * nslot, -1, s);
  hipLaunchKernelGGL(k_inc_emit, dim3(grid_for(nslot, 128)), dim3(128), 0, s, nslot, nt, ns, n, Xn, c.tri.p,
                     c.ref_area.p, cand_off, moved, pair_E, pair_T, prevT, piece_L, inc);
  hipLaunchKernelGGL(k_inc_slot_off, dim3(grid_for(nt + 1, 256)), dim3(256), 0, s, nt, cand_off, e_piece);
  FSI_CHECK_LAUNCH();
  FSI_HIP(hipMemcpyAsync(xold, Xn, 2 * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  c.n_pairs = read_int(inc + 2, s);
  build_rows(c, w, e_piece, pair_T, piece_L, w.flags(), true);
  c.inc_valid = true;
  c.pairs_kept = true;
}

void assemble_coupling(Ctx &c, const double *Xn, bool) {
  if (c.pair == FSI_PAIR_Q2P1DISC) {
    assemble_coupling_q(c, Xn);
    return;
  }
  if (c.cf_mode == FSI_COUPLING_INCREMENTAL) {
    assemble_incremental(c, Xn);
    return;
  }
  GrowWork w{c};
  assemble(c, Xn, w);
  c.pairs_kept = true;
}

// ================================================================ the paper's element pair
// C_f of a Q1 solid against the Q2 fluid on squares (Sec. 4):
//   (C_f)_lj = sum_E int_E N_l(s) phi_j(X^n(s)) ds.
// X^n is bilinear on each reference quadrilateral E, so X^n(E) is the quadrilateral of the
// mapped vertices (it must be strictly convex and counter-clockwise, and inside [0,1]^2).  It is
// clipped against the cells of its bounding box with the arithmetic above (no diagonal) and a
// piece is kept iff its fan area exceeds 5e-11 h^2.  On a piece q the change of variables
// x = X^n(s) gives int_q N_l(xi(x)) phi_j(x) J_s(xi(x)) / J_X(xi(x)) dx, with xi(x) the
// inverse of the bilinear map (Newton's method from the centre of the unit square) and J_s,
// J_X the Jacobian determinants of the reference and the current map.  The rule: the fan of
// q from its vertex 0 and on each fan triangle (A, B, C) the 4 x 4 conical Gauss-Legendre
// points x = A + u (B - A) + u v (C - B), weight 2 |ABC| u w_u w_v: exact for polynomials of
// degree <= 6, so exact whenever X^n is affine on E (the integrand is then of degree 2 + 4).
//
// Pipeline: per quadrilateral the count of kept pieces, a scan, per quadrilateral (a wavefront)
// the pieces (E, cell j n + i) and their 4 x 9 matrices, per solid node one wavefront walking the window
// of lattice nodes its pieces cover (a lane per node, the pieces in a fixed order), and the
// transpose of the triangle pair.
struct GaussPts {
  double u[4], w[4];   // Gauss-Legendre points and weights on [0, 1]
};

__device__ __forceinline__ void load_quad(const double *X, int64_t ns, const int *quad, int64_t e, Pt *P) {
  for (int m = 0; m < 4; ++m) {
    const int v = quad[4 * e + m];
    P[m].x = X[v];
    P[m].y = X[ns + v];
  }
}

__device__ __forceinline__ bool quad_valid(const Pt *P) {
  bool ok = true;
  for (int k = 0; k < 4; ++k) {
    const Pt a = P[(k + 3) & 3], b = P[k], c = P[(k + 1) & 3];
    ok = ok && (b.x - a.x) * (c.y - b.y) - (b.y - a.y) * (c.x - b.x) > 0.0;
    ok = ok && b.x >= 0.0 && b.x <= 1.0 && b.y >= 0.0 && b.y <= 1.0;
  }
  return ok;
}

__device__ __forceinline__ void quad_range(const Pt *P, int n, int &i0, int &i1, int &j0, int &j1) {
  const double xmin = fmin(fmin(P[0].x, P[1].x), fmin(P[2].x, P[3].x));
  const double xmax = fmax(fmax(P[0].x, P[1].x), fmax(P[2].x, P[3].x));
  const double ymin = fmin(fmin(P[0].y, P[1].y), fmin(P[2].y, P[3].y));
  const double ymax = fmax(fmax(P[0].y, P[1].y), fmax(P[2].y, P[3].y));
  const double dn = (double)n;
  i0 = min(max((int)floor(xmin * dn), 0), n - 1);
  i1 = min(max((int)floor(xmax * dn), 0), n - 1);
  j0 = min(max((int)floor(ymin * dn), 0), n - 1);
  j1 = min(max((int)floor(ymax * dn), 0), n - 1);
}

// the piece of quadrilateral P in cell (i, j) into q; its vertex count, 0 when not kept
__device__ __forceinline__ int quad_piece(const Pt *P, int n, int i, int j, Pt *q) {
  Pt a[kMaxPoly], b[kMaxPoly];
  const double dn = (double)n;
  const double xi = (double)i / dn, xi1 = (double)(i + 1) / dn;
  const double yj = (double)j / dn, yj1 = (double)(j + 1) / dn;
  int m = clip_axis(P, 4, a, 0, xi, true);
  m = clip_axis(a, m, b, 0, xi1, false);
  m = clip_axis(b, m, a, 1, yj, true);
  m = clip_axis(a, m, q, 1, yj1, false);
  const double h = 1.0 / dn;
  return (m >= 3 && fan_area(q, m) > 5e-11 * h * h) ? m : 0;
}

__global__ void k_q_count(int64_t nq, int64_t ns, int n, const double *__restrict__ X, const int *__restrict__ quad,
                          int *cnt, int *flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq) return;
  Pt P[4], q[kMaxPoly];
  load_quad(X, ns, quad, e, P);
  if (!quad_valid(P)) {
    atomicOr(flag, DF_MESH);
    cnt[e] = 0;
    return;
  }
  int i0, i1, j0, j1, c = 0;
  quad_range(P, n, i0, i1, j0, j1);
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) c += quad_piece(P, n, i, j, q) ? 1 : 0;
  cnt[e] = c;
}

// bilinear shape functions of the unit square at (xi, eta) and their derivatives
__device__ __forceinline__ void q1_shape(double xi, double eta, double *N, double *Nx, double *Ne) {
  N[0] = (1 - xi) * (1 - eta); N[1] = xi * (1 - eta); N[2] = xi * eta; N[3] = (1 - xi) * eta;
  Nx[0] = -(1 - eta); Nx[1] = 1 - eta; Nx[2] = eta; Nx[3] = -eta;
  Ne[0] = -(1 - xi); Ne[1] = -xi; Ne[2] = xi; Ne[3] = 1 - xi;
}

__device__ __forceinline__ double q1_jac(const Pt *P, const double *Nx, const double *Ne) {
  double a = 0, b = 0, c = 0, d = 0;
  for (int m = 0; m < 4; ++m) {
    a += Nx[m] * P[m].x;
    b += Ne[m] * P[m].x;
    c += Nx[m] * P[m].y;
    d += Ne[m] * P[m].y;
  }
  return a * d - b * c;
}

// (xi, eta) with X(xi, eta) = (x, y) on the bilinear map of P: Newton from (1/2, 1/2) until a
// step below 1e-15 (at most 60 steps)
__device__ __forceinline__ void q1_inverse(const Pt *P, double x, double y, double &xi, double &eta) {
  xi = 0.5;
  eta = 0.5;
  for (int it = 0; it < 60; ++it) {
    double N[4], Nx[4], Ne[4];
    q1_shape(xi, eta, N, Nx, Ne);
    double fx = -x, fy = -y, a = 0, b = 0, c = 0, d = 0;
    for (int m = 0; m < 4; ++m) {
      fx += N[m] * P[m].x;
      fy += N[m] * P[m].y;
      a += Nx[m] * P[m].x;
      b += Ne[m] * P[m].x;
      c += Nx[m] * P[m].y;
      d += Ne[m] * P[m].y;
    }
    const double det = a * d - b * c;
    const double dxi = (d * fx - b * fy) / det, deta = (a * fy - c * fx) / det;
    xi -= dxi;
    eta -= deta;
    if (fmax(fabs(dxi), fabs(deta)) <= 1e-15) break;
  }
}

__device__ __forceinline__ void lagrange2(double t, double *v) {
  v[0] = 2.0 * (t - 0.5) * (t - 1.0);
  v[1] = 4.0 * t * (1.0 - t);
  v[2] = 2.0 * t * (t - 0.5);
}

// One wavefront per quadrilateral: its pieces in cell order (every lane clips the same piece) and
// their matrices L[a][b] = int_q N_a phi_b J_s / J_X (36 per piece, a major): the lanes share the
// 16 (m - 2) points of a piece's fan triangles, then each entry is summed over the wave (a fixed
// butterfly order).
__global__ void __launch_bounds__(kWave) k_q_emit(int64_t nq, int64_t ns, int n, const double *__restrict__ X,
                                                  const double *__restrict__ Xref, const int *__restrict__ quad,
                                                  const int *__restrict__ e_piece, GaussPts g, int *pair_E,
                                                  int *pair_T, double *piece_L) {
  const int64_t e = blockIdx.x;
  if (e >= nq) return;
  const int lane = threadIdx.x;
  Pt P[4], S[4], q[kMaxPoly];
  load_quad(X, ns, quad, e, P);
  load_quad(Xref, ns, quad, e, S);
  if (!quad_valid(P)) return;
  int i0, i1, j0, j1;
  quad_range(P, n, i0, i1, j0, j1);
  const double dn = (double)n;
  int p = e_piece[e];
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      const int m = quad_piece(P, n, i, j, q);
      if (!m) continue;
      double L[36];
      for (int k = 0; k < 36; ++k) L[k] = 0.0;
      for (int it = lane; it < 16 * (m - 2); it += kWave) {
        const int t = 1 + (it >> 4), pu = (it >> 2) & 3, pv = it & 3;
        const Pt A = q[0], B = q[t], C = q[t + 1];
        const double two = (B.x - A.x) * (C.y - A.y) - (C.x - A.x) * (B.y - A.y);
        const double u = g.u[pu], v = g.u[pv];
        const double x = A.x + u * (B.x - A.x) + u * v * (C.x - B.x);
        const double y = A.y + u * (B.y - A.y) + u * v * (C.y - B.y);
        double xi, eta;
        q1_inverse(P, x, y, xi, eta);
        double N[4], Nx[4], Ne[4];
        q1_shape(xi, eta, N, Nx, Ne);
        const double f = g.w[pu] * g.w[pv] * u * two * q1_jac(S, Nx, Ne) / q1_jac(P, Nx, Ne);
        double vx[3], vy[3];
        lagrange2(x * dn - i, vx);
        lagrange2(y * dn - j, vy);
        for (int a = 0; a < 4; ++a) {
          const double fa = f * N[a];
          for (int bb = 0; bb < 3; ++bb)
            for (int ba = 0; ba < 3; ++ba) L[9 * a + ba + 3 * bb] += fa * vx[ba] * vy[bb];
        }
      }
      for (int k = 0; k < 36; ++k) {
        const double v = wave_sum(L[k]);
        if (lane == 0) piece_L[36 * (int64_t)p + k] = v;
      }
      if (lane == 0) {
        pair_E[p] = (int)e;
        pair_T[p] = j * n + i;
      }
      ++p;
    }
}

__device__ __forceinline__ int wave_min_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

// Row l of C_f (one wavefront): the lattice nodes of the cells of its pieces, a lane per node
// in ascending index; each node sums N_a-rows of the pieces of the quadrilaterals around l (in
// element order, then piece order) whose cell holds it.  pass 0: row length; pass 1: entries
// (Dirichlet columns kept with value 0).
__global__ void __launch_bounds__(kWave) k_q_rows(int pass, int64_t ns, int n, const int *__restrict__ n2e_ptr,
                                                  const int *__restrict__ n2e, const int *__restrict__ e_piece,
                                                  const int *__restrict__ pair_T, const double *__restrict__ piece_L,
                                                  int *cnt, const int *__restrict__ rowptr, int *col, double *val) {
  const int64_t l = blockIdx.x;
  if (l >= ns) return;
  const int lane = threadIdx.x;
  const int q0 = n2e_ptr[l], q1 = n2e_ptr[l + 1];
  int imin = n, imax = -1, jmin = n, jmax = -1;
  for (int q = q0; q < q1; ++q) {
    const int e = n2e[q] >> 2;
    for (int p = e_piece[e] + lane; p < e_piece[e + 1]; p += kWave) {
      const int cell = pair_T[p], ci = cell % n, cj = cell / n;
      imin = min(imin, ci);
      imax = max(imax, ci);
      jmin = min(jmin, cj);
      jmax = max(jmax, cj);
    }
  }
  imin = wave_min_i(imin);
  jmin = wave_min_i(jmin);
  imax = wave_max_i(imax);
  jmax = wave_max_i(jmax);
  int total = 0;
  if (imax >= 0) {
    const int I0 = 2 * imin, J0 = 2 * jmin, wx = 2 * (imax - imin) + 3, wn = wx * (2 * (jmax - jmin) + 3);
    const int64_t L = 2 * n + 1;
    const int base = pass ? rowptr[l] : 0;
    for (int w0 = 0; w0 < wn; w0 += kWave) {
      const int w = w0 + lane;
      const int I = I0 + w % wx, J = J0 + w / wx;
      bool hit = false;
      double acc = 0.0;
      if (w < wn)
        for (int q = q0; q < q1; ++q) {
          const int e = n2e[q] >> 2, a = n2e[q] & 3;
          for (int p = e_piece[e]; p < e_piece[e + 1]; ++p) {
            const int cell = pair_T[p];
            const int da = I - 2 * (cell % n), db = J - 2 * (cell / n);
            if (da < 0 || da > 2 || db < 0 || db > 2) continue;
            hit = true;
            if (pass) acc += piece_L[36 * (int64_t)p + 9 * a + da + 3 * db];
          }
        }
      const unsigned long long mask = __ballot(hit);
      if (pass && hit) {
        const int pos = base + total + __popcll(mask & ((1ull << lane) - 1ull));
        col[pos] = (int)(J * L + I);
        val[pos] = (I == 0 || J == 0 || I == 2 * n || J == 2 * n) ? 0.0 : acc;
      }
      total += __popcll(mask);
    }
  }
  if (!pass && lane == 0) cnt[l] = total;
}

// 4-point Gauss-Legendre rule on [0, 1] from its closed form: points 1/2 +- x/2 with
// x = sqrt(3/7 -+ (2/7) sqrt(6/5)) and weights (18 +- sqrt(30)) / 72
static GaussPts gauss4() {
  const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double wa = (18.0 + std::sqrt(30.0)) / 72.0, wb = (18.0 - std::sqrt(30.0)) / 72.0;
  return GaussPts{{0.5 - 0.5 * b, 0.5 - 0.5 * a, 0.5 + 0.5 * a, 0.5 + 0.5 * b}, {wb, wa, wa, wb}};
}

void assemble_coupling_q(Ctx &c, const double *Xn) {
  GrowWork w{c};
  hipStream_t s = c.stream;
  const int64_t nq = c.Nt, ns = c.Ns;
  const int n = c.n;
  c.have_cf = false;
  c.pairs_kept = false;
  c.inc_valid = false;
  int *flag = w.flags();
  int *e_piece = w.work(c.e_piece, nq + 1, "element piece offsets");
  hipLaunchKernelGGL(k_q_count, dim3(grid_for(nq, 128)), dim3(128), 0, s, nq, ns, n, Xn, c.tri.p, e_piece, flag);
  FSI_CHECK_LAUNCH();
  scan_excl(e_piece, e_piece, nq, w.scan(nq), s);
  const int f = read_int(flag, s);
  if (f) fill(flag, 1, 0, s);
  FSI_REQUIRE(!(f & DF_MESH), FSI_E_MESH,
              "X^n maps a solid quadrilateral to one that is not strictly convex and counter-clockwise, or outside [0,1]^2");
  const int npieces = read_int(e_piece + nq, s);
  c.n_pairs = npieces;
  c.n_cand = 0;
  int *pair_E = w.work(c.pair_E, npieces, "piece list");
  int *pair_T = w.work(c.pair_T, npieces, "piece list");
  double *piece_L = w.work(c.piece_L, 36 * (int64_t)npieces, "piece matrices");
  hipLaunchKernelGGL(k_q_emit, dim3((unsigned)nq), dim3(kWave), 0, s, nq, ns, n, Xn, c.ref_xy.p, c.tri.p, e_piece,
                     gauss4(), pair_E, pair_T, piece_L);
  FSI_CHECK_LAUNCH();
  Csr &Cf = c.Cf;
  Cf.nrows = ns;
  Cf.ncols = c.N2;
  Cf.width = 1;
  int *cf_rp = w.out(Cf.rowptr, ns + 1, "the C_f row pointers");
  hipLaunchKernelGGL(k_q_rows, dim3((unsigned)ns), dim3(kWave), 0, s, 0, ns, n, c.n2e_ptr.p, c.n2e.p, e_piece,
                     pair_T, piece_L, cf_rp, nullptr, nullptr, nullptr);
  FSI_CHECK_LAUNCH();
  scan_excl(cf_rp, cf_rp, ns, w.scan(ns), s);
  const int nnz = read_int(cf_rp + ns, s);
  Cf.nnz = nnz;
  int *cf_col = w.out(Cf.col, nnz, "C_f");
  double *cf_val = w.out(Cf.val, nnz, "C_f");
  hipLaunchKernelGGL(k_q_rows, dim3((unsigned)ns), dim3(kWave), 0, s, 1, ns, n, c.n2e_ptr.p, c.n2e.p, e_piece,
                     pair_T, piece_L, nullptr, cf_rp, cf_col, cf_val);
  FSI_CHECK_LAUNCH();
  build_transpose(c, w, nnz, false);
  c.pairs_kept = true;
}

// Coupling storage reserved with the solid (grow-only): row pointers and room for
// kCfPerNode entries per solid node in C_f, C_f^T and their FP32 copies, so that the
// allocation-free assembly can run on a context that has never assembled before.
constexpr int64_t kCfPerNode = 64;
void reserve_coupling(Ctx &c) {
  const size_t e = (size_t)(kCfPerNode * c.Ns);
  c.Cf.rowptr.reserve(c.Ns + 1);
  c.CfT.rowptr.reserve(c.N2 + 1);
  c.Cf.col.reserve(e);
  c.Cf.val.reserve(e);
  c.Cf.val32.reserve(e);
  c.CfT.col.reserve(e);
  c.CfT.val.reserve(e);
  c.CfT.val32.reserve(e);
}

// ---- the allocation-free form: one static work array per GPU
// Every context on a GPU shares that GPU's copy; it keeps the last call's contents.  Host
// code uses the device address taken once per device at set-up, never the symbol itself.
static __device__ __align__(256) unsigned char scratch[FSI_COUPLING_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};
static hipError_t g_scratch_err[kMaxDevices] = {};

// Called by fsi_create with the context's device current; takes the address once per device.
void coupling_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev] || g_scratch_err[dev] != hipSuccess) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_scratch_ptr[dev] = (unsigned char *)p;
  else g_scratch_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

void assemble_coupling_noalloc(Ctx &c, const double *Xn) {
  FSI_REQUIRE(c.device >= 0 && c.device < kMaxDevices, FSI_E_HIP, "context device out of range");
  unsigned char *base = nullptr;
  hipError_t err = hipSuccess;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    base = g_scratch_ptr[c.device];
    err = g_scratch_err[c.device];
  }
  FSI_REQUIRE(base, FSI_E_HIP,
              std::string("no device address of the coupling scratch array: ") +
                  (err != hipSuccess ? hipGetErrorString(err) : "not initialised on this device"));
  ArenaWork w{c, base, (size_t)FSI_COUPLING_SCRATCH_BYTES, 0};
  assemble(c, Xn, w);
}

}  // namespace fsi
