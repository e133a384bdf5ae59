// dmr_adjoint.hip -- reverse-mode (discrete adjoint) kernels of one base step
// of the DMR update: the EM (sub)step of a level (Eqs. (1)-(3) with Mur and
// the TF/SF columns, the window accumulation and, on the patch, the E filter
// and the Eq. (5b) boundary), the fine -> coarse transfer, the window close
// and the continuity step (Eq. (4)) with the density transfers, and the
// Eq. (5a) prolongation of patch growth.
//
// Every kernel is written in gather form: each thread owns the adjoint
// entries it writes and reads whatever it needs, so the results do not
// depend on scheduling.  Forward values come from the recorded tape; the
// E filter and the clamp of the continuity step are recomputed with the
// forward's own expressions.
//
// Notation: for a forward statement y = f(x), lam_x += (df/dx)^T lam_y.
// EM step in the scaled variables of the forward (H~ = eta0 Hz, J~ =
// (dt/eps0) J, k = kn n_e):
//   H'  = H - S[(Ey_{i+1}-Ey_i) - (Ex_{j+1}-Ex_j)]
//   E'  = [(1-k)E + S dH' - c1 J]/(1+k),  J' = aJ + 2k(E+E')
// With G = (lam E' total) + 2k lam J' and g = G/(1+k):
//   lam E += (1-k) g + 2k lam J',   lam J = a lam J' - c1 g,
//   lam k = (E+E')(2 lam J' - g),   lam H' += S g on the two cells of dH'.
#include "dmr_kernels.h"

namespace dmr {

namespace {

constexpr int kAT = 64, kAR = kThreads / 64;  // node tile: 64 x 4

__device__ inline size_t at(int i, int j, int p) { return (size_t)j * p + i; }

// weight of the window sum of a node w.r.t. one squared edge: 1/2 where the
// node has two edges along that axis, 1 where it has one
__device__ inline float wwin(int q, int lo, int hi) { return (q > lo && q < hi) ? 0.5f : 1.f; }

// ---- gather helpers ----------------------------------------------------------
// Every thread first loads all the values it needs from clamped (always
// valid) addresses, then computes; entries that do not exist are discarded
// by selects.  (Loads under conditions would each wait for memory.)
struct Reg {
  int L, B, R, T, p;
  __device__ size_t o(int a, int b) const {
    a = a < L ? L : (a > R ? R : a);
    b = b < B ? B : (b > T ? T : b);
    return (size_t)b * p + a;
  }
  __device__ float ld(const float* q, int a, int b) const { return q[o(a, b)]; }
  __device__ bool ex(int a, int b) const { return a >= L && a < R && b >= B && b <= T; }
  __device__ bool ey(int a, int b) const { return a >= L && a <= R && b >= B && b < T; }
  __device__ bool hz(int a, int b) const { return a >= L && a < R && b >= B && b < T; }
};

__device__ inline float lap5a(float c, float l, float r, float d, float u) {
  return l + r + d + u - 4.f * c;
}

// 13-point diamond around (i, j): slot of offset (a, b), |a| + |b| <= 2
__device__ constexpr int dmd(int a, int b) {
  return (a == 0 && b == 0) ? 0 : (a == -1 && b == 0) ? 1 : (a == 1 && b == 0) ? 2
       : (a == 0 && b == -1) ? 3 : (a == 0 && b == 1) ? 4 : (a == -2 && b == 0) ? 5
       : (a == 2 && b == 0) ? 6 : (a == 0 && b == -2) ? 7 : (a == 0 && b == 2) ? 8
       : (a == -1 && b == -1) ? 9 : (a == 1 && b == -1) ? 10 : (a == -1 && b == 1) ? 11 : 12;
}

template <class OK>
__device__ inline void load13(const Reg& g, const float* q, int i, int j, float v[13]) {
#pragma unroll
  for (int b = -2; b <= 2; b++)
#pragma unroll
    for (int a = -2; a <= 2; a++)
      if ((a < 0 ? -a : a) + (b < 0 ? -b : b) <= 2) v[dmd(a, b)] = g.ld(q, i + a, j + b);
}

// L(L(v)) at (i, j) from the diamond, neighbours outside the component's
// grid replaced by the centre value (the forward filter's rule)
template <class OK>
__device__ inline float ll13(const float v[13], int i, int j, OK ok) {
  auto lapP = [&](int a, int b) {
    const float c = v[dmd(a, b)];
    return lap5a(c, ok(i + a - 1, j + b) ? v[dmd(a - 1, b)] : c,
                 ok(i + a + 1, j + b) ? v[dmd(a + 1, b)] : c,
                 ok(i + a, j + b - 1) ? v[dmd(a, b - 1)] : c,
                 ok(i + a, j + b + 1) ? v[dmd(a, b + 1)] : c);
  };
  const float c = lapP(0, 0);
  return lap5a(c, ok(i - 1, j) ? lapP(-1, 0) : c, ok(i + 1, j) ? lapP(1, 0) : c,
               ok(i, j - 1) ? lapP(0, -1) : c, ok(i, j + 1) ? lapP(0, 1) : c);
}

// ---------------------------------------------------------------------------
// EM adjoint of one (sub)step of a level, one launch per (sub)step.  A block
// owns a kAdjTX x kAdjTY tile of node positions (i, j) (cell (i, j), x-edge
// (i, j), y-edge (i, j), node (i, j)) and runs three phases through LDS:
//   1. per edge over the tile grown by H1: G, g = G/(1+k) and lam k
//      (boundary edges keep G: Mur feeds the interior neighbour and the old
//      values; on the patch it is the lam of the coarse-driven value);
//   2. per position over the tile grown by H2: lam of H' at the cells, lam E
//      and lam J entering, lam n at the nodes, source-column sums;
//   3. (patch) the E filter transposed: E~ = E - gamma P L(L(E)) with P the
//      filtered edges and L symmetric, so lam E = lam E~ - gamma L(L(P lam E~)).
// Halo values are recomputed, never exchanged; lam E and lam J are read
// from one buffer and written to another, so no block reads what another
// block writes in the same launch.
// ---------------------------------------------------------------------------
// Tiles: patch 16 x 5 positions (phase-1 region 22 x 11, phase-2 20 x 9),
// base level 32 x 5 (34 x 7, phase 2 = the tile); 256 threads, so every
// phase is one position per thread and all of a thread's loads for both
// phases are issued before any arithmetic.  On a 512 x 256 base level the
// sweep is latency-bound: small blocks spread over every CU beat large
// ones despite the recomputed halos (1024-thread 32 x 28 / 32 x 16 tiles
// took 37% longer per reverse step, 512-thread ones 10%).
template <bool FINE> struct AdjTile {
  static constexpr int TX = FINE ? 16 : 32, TY = 5, NT = 256;
  static constexpr int H1 = FINE ? 3 : 1, H2 = FINE ? 2 : 0;
  static constexpr int W1 = TX + 2 * H1, N1 = TY + 2 * H1;
  static constexpr int W2 = TX + 2 * H2, N2 = TY + 2 * H2;
  static_assert(W1 * N1 <= NT && W2 * N2 <= NT, "one position per thread");
};

// coarse entity of fine position (i, j) of the patch region g
__device__ inline size_t coarse_of(const AdjEMArgs& A, const Reg& g, int i, int j) {
  const int a = i < g.L ? g.L : (i > g.R ? g.R : i), b = j < g.B ? g.B : (j > g.T ? g.T : j);
  return (size_t)(b >> 1) * A.cpitch + (a >> 1);
}

// Folded fine -> coarse transfer (patch, last substep): a fine entity gets
// the coarse lam of the entity it was averaged into: Hz 1/4 of the cell mean
// x 1/2 of the two half levels, E 1/2 of the edge mean, J~ the sum.
// x-edges (X) on even rows strictly inside, y-edges on even columns.
template <bool X>
__device__ inline bool fold_edge(const AdjEMArgs& A, int i, int j) {
  const int q = X ? j : i, q0 = X ? A.J0 : A.I0, q1 = X ? A.J1 : A.I1;
  return (q & 1) == 0 && (q >> 1) > q0 && (q >> 1) < q1;
}
// base level: coarse entities strictly inside the patch (their lam went to it)
__device__ inline bool inside_hz(const AdjEMArgs& A, int i, int j) {
  return A.has_patch && i >= A.I0 && i < A.I1 && j >= A.J0 && j < A.J1;
}
__device__ inline bool inside_ex(const AdjEMArgs& A, int i, int j) {
  return A.has_patch && i >= A.I0 && i < A.I1 && j > A.J0 && j < A.J1;
}
__device__ inline bool inside_ey(const AdjEMArgs& A, int i, int j) {
  return A.has_patch && i > A.I0 && i < A.I1 && j >= A.J0 && j < A.J1;
}

// Eq. (5b) transposed at coarse edge (i, j) of a patch boundary line: fine
// boundary g of one substep weighted 1/4, 3/4, 3/4, 1/4 in space.  Split in
// the four (clamped) loads and the sum, zero off the lines.
template <bool X>
__device__ inline void cfb_load(const AdjEMArgs& A, const float* gf, int i, int j, float v[4]) {
  const int c = X ? i : j, line = X ? j : i;
  const int l0 = X ? A.J0 : A.I0, l1 = X ? A.J1 : A.I1;
  const int lo = X ? A.fL : A.fB, hi = X ? A.fR : A.fT;
  const int f = 2 * (line < l0 ? l0 : (line > l1 ? l1 : line));
#pragma unroll
  for (int q = 0; q < 4; q++) {
    int fc = 2 * c - 1 + q;
    fc = fc < lo ? lo : (fc > hi ? hi : fc);
    v[q] = X ? gf[(size_t)f * A.fpitch + fc] : gf[(size_t)fc * A.fpitch + f];
  }
}
// G of patch substep 1 at the fine boundary edges of coarse edge (i, j):
// lam E + the window terms + 2 k lam J, the patch kernel's expression for a
// boundary edge (substep 1 has no fine -> coarse fold)
template <bool X>
__device__ inline void cfb_g1(const AdjEMArgs& A, int i, int j, float v[4]) {
  const int c = X ? i : j, line = X ? j : i;
  const int l0 = X ? A.J0 : A.I0, l1 = X ? A.J1 : A.I1;
  const int lo = X ? A.fL : A.fB, hi = X ? A.fR : A.fT;
  const int f = 2 * (line < l0 ? l0 : (line > l1 ? l1 : line));
  const int p = A.fpitch;
  float le[4], en[4], a0[4], a1[4], n0[4], n1[4], lj[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    int fc = 2 * c - 1 + q;
    fc = fc < lo ? lo : (fc > hi ? hi : fc);
    const int fc1 = fc + 1 > hi ? hi : fc + 1;
    const size_t o = X ? (size_t)f * p + fc : (size_t)fc * p + f;
    const size_t o1 = X ? (size_t)f * p + fc1 : (size_t)fc1 * p + f;
    le[q] = X ? A.s1ex[o] : A.s1ey[o];
    lj[q] = X ? A.s1jx[o] : A.s1jy[o];
    en[q] = X ? A.s1exo[o] : A.s1eyo[o];
    a0[q] = A.s1acc[o]; a1[q] = A.s1acc[o1];
    n0[q] = A.s1n[o]; n1[q] = A.s1n[o1];
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int fc = 2 * c - 1 + q;
    const float kap = A.s1kn * (0.5f * (n0[q] + n1[q]));
    const float tot = le[q] + 2.f * en[q] * (wwin(fc, lo, hi) * a0[q] + wwin(fc + 1, lo, hi) * a1[q]);
    v[q] = tot + 2.f * kap * lj[q];
  }
}

template <bool X>
__device__ inline float cfb_sum(const AdjEMArgs& A, const float v[4], int i, int j) {
  const int c = X ? i : j, line = X ? j : i;
  const int l0 = X ? A.J0 : A.I0, l1 = X ? A.J1 : A.I1, c0 = X ? A.I0 : A.J0, c1 = X ? A.I1 : A.J1;
  const int lo = X ? A.fL : A.fB, hi = X ? A.fR : A.fT;
  const float w[4] = {0.25f, 0.75f, 0.75f, 0.25f};
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int fc = 2 * c - 1 + q;
    s += (fc >= lo && fc < hi) ? w[q] * v[q] : 0.f;
  }
  const bool on = (line == l0 || line == l1) && c >= c0 - 1 && c <= c1;
  return on ? s : 0.f;
}

// values phase 1 needs at position (i, j)
struct P1In {
  float xle, xlj, yle, ylj;            // lam E, J leaving
  float rxe, rye, rxj, ryj;            // patch, last substep: coarse lam (fold)
  float xen, xeo, yen, yeo;            // E leaving / entering
  float a00, a10, a01;                 // lam acc at the end nodes
  float n00, n10, n01;                 // density at the end nodes
  float mx[7], my[7];                  // base: the Mur partner edges
  float dx[13], dy[13];                // patch: E entering on the filter's diamond
  float c1x[4], c2x[4], c1y[4], c2y[4];  // base: patch g for Eq. (5b) transposed
};

// mur / cfb: the block's phase-1 region reaches a Mur partner row or
// column / a patch boundary line (uniform per block)
template <bool FINE>
__device__ inline void p1_load(const AdjEMArgs& A, const Reg& g, int i, int j, P1In& v,
                               bool mur, bool cfb) {
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  v.xle = g.ld(A.lex, i, j); v.xlj = g.ld(A.ljx, i, j);
  v.yle = g.ld(A.ley, i, j); v.ylj = g.ld(A.ljy, i, j);
  v.xen = g.ld(A.exo, i, j); v.xeo = g.ld(A.exi, i, j);
  v.yen = g.ld(A.eyo, i, j); v.yeo = g.ld(A.eyi, i, j);
  v.a00 = g.ld(A.lacc, i, j); v.a10 = g.ld(A.lacc, i + 1, j); v.a01 = g.ld(A.lacc, i, j + 1);
  v.n00 = g.ld(A.n, i, j); v.n10 = g.ld(A.n, i + 1, j); v.n01 = g.ld(A.n, i, j + 1);
  if constexpr (FINE) {
    auto ex_ok = [=](int a, int b) { return g.ex(a, b); };
    auto ey_ok = [=](int a, int b) { return g.ey(a, b); };
    load13<decltype(ex_ok)>(g, A.exi, i, j, v.dx);
    load13<decltype(ey_ok)>(g, A.eyi, i, j, v.dy);
    v.rxe = v.rye = v.rxj = v.ryj = 0.f;
    if (A.rex) {
      const size_t c = coarse_of(A, g, i, j);
      v.rxe = A.rex[c]; v.rye = A.rey[c]; v.rxj = A.rjx[c]; v.ryj = A.rjy[c];
    }
  } else {
    if (mur) {
      // Mur partners (own edge where there is none: a cache hit, never used)
      const int jb = (j == B + 1) ? B : (j == T - 1 ? T : j);
      const int ib = (i == L + 1) ? L : (i == R - 1 ? R : i);
      v.mx[0] = g.ld(A.lex, i, jb); v.mx[1] = g.ld(A.exo, i, jb); v.mx[2] = g.ld(A.lacc, i, jb);
      v.mx[3] = g.ld(A.lacc, i + 1, jb); v.mx[4] = g.ld(A.n, i, jb); v.mx[5] = g.ld(A.n, i + 1, jb);
      v.mx[6] = g.ld(A.ljx, i, jb);
      v.my[0] = g.ld(A.ley, ib, j); v.my[1] = g.ld(A.eyo, ib, j); v.my[2] = g.ld(A.lacc, ib, j);
      v.my[3] = g.ld(A.lacc, ib, j + 1); v.my[4] = g.ld(A.n, ib, j); v.my[5] = g.ld(A.n, ib, j + 1);
      v.my[6] = g.ld(A.ljy, ib, j);
    } else {
#pragma unroll
      for (int q = 0; q < 7; q++) { v.mx[q] = 0.f; v.my[q] = 0.f; }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) { v.c1x[q] = v.c2x[q] = v.c1y[q] = v.c2y[q] = 0.f; }
    if (cfb) {
      cfb_g1<true>(A, i, j, v.c1x); cfb_load<true>(A, A.g2x, i, j, v.c2x);
      cfb_g1<false>(A, i, j, v.c1y); cfb_load<false>(A, A.g2y, i, j, v.c2y);
    }
  }
}

// phase 1 at position (i, j): g and lam k of x-edge (i, j) and y-edge (i, j)
// (zero where the edge does not exist); base level: px, py = the lam of the
// coarse E entering the step from Eq. (5b)
template <bool FINE>
__device__ inline void p1_compute(const AdjEMArgs& A, const Reg& g, int i, int j, P1In& v,
                                  float& gx, float& kx, float& gy, float& ky, float& px,
                                  float& py) {
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  auto ex_ok = [=](int a, int b) { return g.ex(a, b); };
  auto ey_ok = [=](int a, int b) { return g.ey(a, b); };
  float xle = v.xle, xlj = v.xlj, yle = v.yle, ylj = v.ylj;
  px = 0.f; py = 0.f;
  if constexpr (FINE) {
    if (A.rex) {
      if (fold_edge<true>(A, i, j)) { xle += 0.5f * v.rxe; xlj += v.rxj; }
      if (fold_edge<false>(A, i, j)) { yle += 0.5f * v.rye; ylj += v.ryj; }
    }
  } else {
    if (inside_ex(A, i, j)) { xle = 0.f; xlj = 0.f; }
    if (inside_ey(A, i, j)) { yle = 0.f; ylj = 0.f; }
    if (A.has_patch) {
      // Eq. (5b) in time: substep m takes m/2 of E^{n+1} and 1 - m/2 of E^n
      const float s1x = cfb_sum<true>(A, v.c1x, i, j), s2x = cfb_sum<true>(A, v.c2x, i, j);
      const float s1y = cfb_sum<false>(A, v.c1y, i, j), s2y = cfb_sum<false>(A, v.c2y, i, j);
      xle = (xle + 1.f * s2x) + 0.5f * s1x;
      yle = (yle + 1.f * s2y) + 0.5f * s1y;
      px = (0.f + 0.f * s2x) + 0.5f * s1x;
      py = (0.f + 0.f * s2y) + 0.5f * s1y;
    }
  }
  auto kapf = [&](float a, float b) { return A.kn * (0.5f * (a + b)); };
  gx = 0.f; kx = 0.f; gy = 0.f; ky = 0.f;
  if (ex_ok(i, j)) {
    const float kap = kapf(v.n00, v.n10);
    const bool bnd = (j == B || j == T);
    float eo = v.xeo;
    if (FINE && A.gamma > 0.f && !bnd) eo -= A.gamma * ll13(v.dx, i, j, ex_ok);
    // own lam plus the window: acc at both end nodes (1/2 where a node has two x-edges)
    float tot = xle + 2.f * v.xen * (wwin(i, L, R) * v.a00 + wwin(i + 1, L, R) * v.a10);
    if (!bnd) {
      if (!FINE && A.bc_y == kBcMur && (j == B + 1 || j == T - 1)) {
        const float* m = v.mx;
        const float ab = m[0] + 2.f * m[1] * (wwin(i, L, R) * m[2] + wwin(i + 1, L, R) * m[3]);
        tot += A.cmur * (ab + 2.f * kapf(m[4], m[5]) * m[6]);
      }
      gx = (tot + 2.f * kap * xlj) * __builtin_amdgcn_rcpf(1.f + kap);  // the forward's factor
      kx = (eo + v.xen) * (2.f * xlj - gx);
    } else {
      gx = tot + 2.f * kap * xlj;
      kx = 2.f * (eo + v.xen) * xlj;
    }
  }
  if (ey_ok(i, j)) {
    const float kap = kapf(v.n00, v.n01);
    const bool bnd = (i == L || i == R);
    float eo = v.yeo;
    if (FINE && A.gamma > 0.f && !bnd) eo -= A.gamma * ll13(v.dy, i, j, ey_ok);
    float tot = yle + 2.f * v.yen * (wwin(j, B, T) * v.a00 + wwin(j + 1, B, T) * v.a01);
    if (!bnd) {
      if (!FINE && A.bc_x == kBcMur && (i == L + 1 || i == R - 1)) {
        const float* m = v.my;
        const float ab = m[0] + 2.f * m[1] * (wwin(j, B, T) * m[2] + wwin(j + 1, B, T) * m[3]);
        tot += A.cmur * (ab + 2.f * kapf(m[4], m[5]) * m[6]);
      }
      gy = (tot + 2.f * kap * ylj) * __builtin_amdgcn_rcpf(1.f + kap);
      ky = (eo + v.yen) * (2.f * ylj - gy);
    } else {
      gy = tot + 2.f * kap * ylj;
      ky = 2.f * (eo + v.yen) * ylj;
    }
  }
}

// values phase 2 needs at position (i, j)
struct P2In {
  float h00, h0m, hm0;     // lam Hz leaving at cells (i,j), (i,j-1), (i-1,j)
  float r00, r0m, rm0;     // patch, last substep: coarse lam Hz of those cells (fold)
  float ljx, ljy, rjx, rjy;
  float n00, n10, n01, ln0, hxv;
};

template <bool FINE>
__device__ inline void p2_load(const AdjEMArgs& A, const Reg& g, int i, int j, P2In& v) {
  v.h00 = g.ld(A.lhz_in, i, j); v.h0m = g.ld(A.lhz_in, i, j - 1); v.hm0 = g.ld(A.lhz_in, i - 1, j);
  v.ljx = g.ld(A.ljx, i, j); v.ljy = g.ld(A.ljy, i, j);
  v.n00 = g.ld(A.n, i, j); v.n10 = g.ld(A.n, i + 1, j); v.n01 = g.ld(A.n, i, j + 1);
  v.ln0 = g.ld(A.ln, i, j);
  v.r00 = v.r0m = v.rm0 = v.rjx = v.rjy = v.hxv = 0.f;
  if constexpr (FINE) {
    if (A.rhz) {
      v.r00 = A.rhz[coarse_of(A, g, i, j)];
      v.r0m = A.rhz[coarse_of(A, g, i, j - 1)];
      v.rm0 = A.rhz[coarse_of(A, g, i - 1, j)];
      const size_t c = coarse_of(A, g, i, j);
      v.rjx = A.rjx[c]; v.rjy = A.rjy[c];
    }
  } else {
    if (A.hz_extra) v.hxv = g.ld(A.hz_extra, i, j);
  }
}

template <bool FINE>
__device__ __forceinline__ void adj_em_tile(const AdjEMArgs& A, int bx, int by) {
  using Tl = AdjTile<FINE>;
  constexpr int TX = Tl::TX, TY = Tl::TY, H1 = Tl::H1, H2 = Tl::H2;
  constexpr int W1 = Tl::W1, N1 = Tl::N1, W2 = Tl::W2, N2 = Tl::N2;
  __shared__ float sgx[N1][W1], sgy[N1][W1], skx[N1][W1], sky[N1][W1];
  __shared__ float spx[FINE ? 1 : N1][FINE ? 1 : W1], spy[FINE ? 1 : N1][FINE ? 1 : W1];
  __shared__ float stx[FINE ? N2 : 1][FINE ? W2 : 1], sty[FINE ? N2 : 1][FINE ? W2 : 1];
  const Reg g{A.L, A.B, A.R, A.T, A.pitch};
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const int i0 = L + bx * TX, j0 = B + by * TY;
  const int tid = threadIdx.x;
  const float S = A.S;
  const bool filt = FINE && A.gamma > 0.f;

  // this thread's positions: phase 1 (tile grown by H1), phase 2 (by H2)
  const bool a1 = tid < N1 * W1, a2 = tid < N2 * W2;
  const int c1i = a1 ? tid % W1 : 0, c1j = a1 ? tid / W1 : 0;
  const int c2i = a2 ? tid % W2 : 0, c2j = a2 ? tid / W2 : 0;
  const int i1 = i0 - H1 + c1i, j1 = j0 - H1 + c1j;
  const int i = i0 - H2 + c2i, j = j0 - H2 + c2j;

  // -- every load of both phases ------------------------------------------------
  // (block-uniform: Mur partner rows / columns, patch boundary lines)
  const int rl = i0 - H1, rr = i0 + TX + H1 - 1, rb = j0 - H1, rt = j0 + TY + H1 - 1;
  auto span = [](int lo, int hi, int a, int b) { return hi >= a && lo <= b; };
  const bool mur = !FINE && (span(rb, rt, B + 1, B + 1) || span(rb, rt, T - 1, T - 1) ||
                             span(rl, rr, L + 1, L + 1) || span(rl, rr, R - 1, R - 1));
  const bool cfb = !FINE && A.has_patch &&
                   (((span(rb, rt, A.J0, A.J0) || span(rb, rt, A.J1, A.J1)) &&
                     span(rl, rr, A.I0 - 1, A.I1)) ||
                    ((span(rl, rr, A.I0, A.I0) || span(rl, rr, A.I1, A.I1)) &&
                     span(rb, rt, A.J0 - 1, A.J1)));
  P1In v1;
  p1_load<FINE>(A, g, i1, j1, v1, mur, cfb);
  P2In v2;
  p2_load<FINE>(A, g, i, j, v2);

  // -- phase 1 --------------------------------------------------------------------
  if (a1) {
    float gx, kx, gy, ky, px, py;
    p1_compute<FINE>(A, g, i1, j1, v1, gx, kx, gy, ky, px, py);
    sgx[c1j][c1i] = gx; skx[c1j][c1i] = kx;
    sgy[c1j][c1i] = gy; sky[c1j][c1i] = ky;
    if constexpr (!FINE) { spx[c1j][c1i] = px; spy[c1j][c1i] = py; }
  }
  __syncthreads();
  auto GX = [&](int a, int b) { return sgx[b - j0 + H1][a - i0 + H1]; };
  auto GY = [&](int a, int b) { return sgy[b - j0 + H1][a - i0 + H1]; };
  auto KX = [&](int a, int b) { return skx[b - j0 + H1][a - i0 + H1]; };
  auto KY = [&](int a, int b) { return sky[b - j0 + H1][a - i0 + H1]; };

  // -- phase 2 --------------------------------------------------------------------
  if (a2) {
    const bool own = c2i >= H2 && c2i < H2 + TX && c2j >= H2 && c2j < H2 + TY && i <= R && j <= T;
    float h00 = v2.h00, h0m = v2.h0m, hm0 = v2.hm0, ljx = v2.ljx, ljy = v2.ljy, hxv = v2.hxv;
    float pxv = 0.f, pyv = 0.f;
    if constexpr (FINE) {
      if (A.rhz) {
        h00 = h00 + 0.125f * v2.r00;
        h0m = h0m + 0.125f * v2.r0m;
        hm0 = hm0 + 0.125f * v2.rm0;
        hxv = 0.125f * v2.r00;
        if (fold_edge<true>(A, i, j)) ljx += v2.rjx;
        if (fold_edge<false>(A, i, j)) ljy += v2.rjy;
      }
    } else {
      if (inside_hz(A, i, j)) h00 = 0.f;
      if (inside_hz(A, i, j - 1)) h0m = 0.f;
      if (inside_hz(A, i - 1, j)) hm0 = 0.f;
      if (inside_ex(A, i, j)) ljx = 0.f;
      if (inside_ey(A, i, j)) ljy = 0.f;
      pxv = spx[j - j0 + H1][i - i0 + H1];
      pyv = spy[j - j0 + H1][i - i0 + H1];
    }
    // g of interior edges (boundary E' does not depend on H')
    auto xi = [&](int a, int b) { return (b == B || b == T) ? 0.f : GX(a, b); };
    auto yi = [&](int a, int b) { return (a == L || a == R) ? 0.f : GY(a, b); };
    // lam of H' at a cell: its own plus the curl terms of the four edges
    const float hc00 = h00 + S * (xi(i, j) - xi(i, j + 1)) + S * (yi(i + 1, j) - yi(i, j));
    const float hc0m = h0m + S * (xi(i, j - 1) - xi(i, j)) + S * (yi(i + 1, j - 1) - yi(i, j - 1));
    const float hcm0 = hm0 + S * (xi(i - 1, j) - xi(i - 1, j + 1)) + S * (yi(i, j) - yi(i - 1, j));
    const size_t o = g.o(i, j);
    float tex = 0.f, tey = 0.f;
    if (g.hz(i, j) && own) {
      if (A.src_e && i == A.is - 1) A.src_e[j] = S * hc00;
      A.lhz_out[o] = hc00 + hxv;
      if (!FINE && A.hz_extra) A.hz_extra[o] = 0.f;
    }
    if (g.ex(i, j)) {
      const float gxv = GX(i, j);
      const float kap = A.kn * (0.5f * (v2.n00 + v2.n10));
      float le = (g.hz(i, j - 1) ? S * hc0m : 0.f) - (g.hz(i, j) ? S * hc00 : 0.f);
      const bool bnd = (j == B || j == T);
      float ljn;
      if (!bnd) {
        le += (1.f - kap) * gxv + 2.f * kap * ljx;
        ljn = A.a * ljx - A.c1 * gxv;
        if (!FINE && A.bc_y == kBcMur) {
          if (j == B + 1) le += GX(i, B);
          if (j == T - 1) le += GX(i, T);
        }
      } else {
        le += 2.f * kap * ljx;
        if (!FINE && A.bc_y == kBcMur) le -= A.cmur * gxv;
        ljn = A.a * ljx;
      }
      le += pxv;
      tex = le;
      if (own) {
        if (!filt) A.lex_o[o] = le;
        A.ljx_o[o] = ljn;
        if (FINE) A.gx[o] = gxv;
      }
    }
    if (g.ey(i, j)) {
      const float gyv = GY(i, j);
      const float kap = A.kn * (0.5f * (v2.n00 + v2.n01));
      float le = (g.hz(i, j) ? S * hc00 : 0.f) - (g.hz(i - 1, j) ? S * hcm0 : 0.f);
      const bool bnd = (i == L || i == R);
      float ljn;
      if (!bnd) {
        if (own && A.src_h && i == A.is) A.src_h[j] = S * gyv;
        le += (1.f - kap) * gyv + 2.f * kap * ljy;
        ljn = A.a * ljy - A.c1 * gyv;
        if (!FINE && A.bc_x == kBcMur) {
          if (i == L + 1) le += GY(L, j);
          if (i == R - 1) le += GY(R, j);
        }
      } else {
        le += 2.f * kap * ljy;
        if (!FINE && A.bc_x == kBcMur) le -= A.cmur * gyv;
        ljn = A.a * ljy;
      }
      le += pyv;
      tey = le;
      if (own) {
        if (!filt) A.ley_o[o] = le;
        A.ljy_o[o] = ljn;
        if (FINE) A.gy[o] = gyv;
      }
    }
    if (own) {
      // node: k of the (up to four) edges that average this node's density
      float sk = 0.f;
      if (g.ex(i - 1, j)) sk += KX(i - 1, j);
      if (g.ex(i, j)) sk += KX(i, j);
      if (g.ey(i, j - 1)) sk += KY(i, j - 1);
      if (g.ey(i, j)) sk += KY(i, j);
      A.ln[o] = v2.ln0 + 0.5f * A.kn * sk;
    }
    if constexpr (FINE) {
      stx[c2j][c2i] = tex;
      sty[c2j][c2i] = tey;
    }
  }

  // -- phase 3 (patch): E filter transposed ---------------------------------------
  if constexpr (FINE) {
    if (!filt) return;
    __syncthreads();
    auto ex_ok = [=](int a, int b) { return g.ex(a, b); };
    auto ey_ok = [=](int a, int b) { return g.ey(a, b); };
    if (tid >= TX * TY) return;
    const int ii = i0 + tid % TX, jj = j0 + tid / TX;
    if (ii > R || jj > T) return;
    // P lam E~ on the diamond: only filtered edges (not the boundary ones)
    float tx[13], ty[13];
#pragma unroll
    for (int b = -2; b <= 2; b++)
#pragma unroll
      for (int a = -2; a <= 2; a++)
        if ((a < 0 ? -a : a) + (b < 0 ? -b : b) <= 2) {
          const int q = dmd(a, b);
          const float vx = stx[jj - j0 + H2 + b][ii - i0 + H2 + a];
          const float vy = sty[jj - j0 + H2 + b][ii - i0 + H2 + a];
          tx[q] = (jj + b == B || jj + b == T) ? 0.f : vx;
          ty[q] = (ii + a == L || ii + a == R) ? 0.f : vy;
        }
    const size_t o = g.o(ii, jj);
    const float tex = stx[jj - j0 + H2][ii - i0 + H2], tey = sty[jj - j0 + H2][ii - i0 + H2];
    if (g.ex(ii, jj)) A.lex_o[o] = tex - A.gamma * ll13(tx, ii, jj, ex_ok);
    if (g.ey(ii, jj)) A.ley_o[o] = tey - A.gamma * ll13(ty, ii, jj, ey_ok);
  }
}

// ---------------------------------------------------------------------------
// Eq. (5a) prolongation of growth, transposed: each coarse entity gathers
// the lam of the newly covered fine entities that interpolated from it.
// ---------------------------------------------------------------------------
// weight of coarse index a in the 1-D linear interpolation at quarter-unit
// position U4 (the forward skips zero weights)
__device__ inline float w1(int U4, int a) {
  const int c = U4 >> 2;
  const float f = (U4 & 3) * 0.25f;
  if (c == a) return 1.f - f;
  if (c + 1 == a && f != 0.f) return f;
  return 0.f;
}

__global__ __launch_bounds__(kThreads) void k_adj_grow(AdjGrowArgs A) {
  const int a = A.cL + blockIdx.x * kAT + (threadIdx.x % kAT);
  const int b = A.cB + blockIdx.y * kAR + (threadIdx.x / kAT);
  if (a > A.cR || b > A.cT) return;
  const int p = A.pitch;
  const bool old = A.oR > A.oL;
  auto in_old = [&](int i, int j, int hx, int hy) {
    return old && i >= A.oL && i <= A.oR - hx && j >= A.oB && j <= A.oT - hy;
  };
  auto in_new = [&](int i, int j, int hx, int hy) {
    return i >= A.L && i <= A.R - hx && j >= A.B && j <= A.T - hy;
  };
  // sum over fine entities (offsets dx, dy of their quarter positions)
  auto gather = [&](const float* f, int hx, int hy, int du, int dv) {
    float s = 0.f;
    for (int j = 2 * b - 2; j <= 2 * b + 2; j++) {
      const float wv = w1(2 * j + dv, b);
      if (wv == 0.f) continue;
      for (int i = 2 * a - 2; i <= 2 * a + 2; i++) {
        const float wu = w1(2 * i + du, a);
        if (wu == 0.f) continue;
        if (!in_new(i, j, hx, hy) || in_old(i, j, hx, hy)) continue;
        s += wu * wv * f[at(i, j, p)];
      }
    }
    return s;
  };
  const size_t co = at(a, b, A.cpitch);
  if (a < A.cNX && b < A.cNY) {
    const float s = gather(A.lhz, 1, 1, -1, -1);
    A.chz[co] += 1.25f * s;
    A.chz_prev[co] += (1.f - 1.25f) * s;
  }
  if (a < A.cNX) {
    A.cex[co] += gather(A.lex, 1, 0, -1, 0);
    A.cjx[co] += 0.5f * gather(A.ljx, 1, 0, -1, 0);
  }
  if (b < A.cNY) {
    A.cey[co] += gather(A.ley, 0, 1, 0, -1);
    A.cjy[co] += 0.5f * gather(A.ljy, 0, 1, 0, -1);
  }
  if (A.with_n) A.cn[co] += gather(A.ln, 0, 0, 0, 0);
  A.cacc[co] += gather(A.lacc, 0, 0, 0, 0);
  for (int s = 0; s < kRing; s++)
    A.cring[(size_t)s * A.cplane + co] += gather(A.lring + (size_t)s * A.plane, 0, 0, 0, 0);
}

// the newly covered fine entities had no value before the growth: clear
// their lam once the coarse side has gathered it
__global__ __launch_bounds__(kThreads) void k_adj_grow_clear(AdjGrowArgs A, float* lhz,
                                                             float* lex, float* ley,
                                                             float* ljx, float* ljy,
                                                             float* ln, float* lacc,
                                                             float* lring) {
  const int i = A.L + blockIdx.x * kAT + (threadIdx.x % kAT);
  const int j = A.B + blockIdx.y * kAR + (threadIdx.x / kAT);
  if (i > A.R || j > A.T) return;
  const bool old = A.oR > A.oL;
  auto fresh = [&](int hx, int hy) {
    if (i > A.R - hx || j > A.T - hy) return false;
    return !(old && i >= A.oL && i <= A.oR - hx && j >= A.oB && j <= A.oT - hy);
  };
  const size_t o = at(i, j, A.pitch);
  if (fresh(1, 1)) lhz[o] = 0.f;
  if (fresh(1, 0)) { lex[o] = 0.f; ljx[o] = 0.f; }
  if (fresh(0, 1)) { ley[o] = 0.f; ljy[o] = 0.f; }
  if (fresh(0, 0)) {
    if (A.with_n) ln[o] = 0.f;
    lacc[o] = 0.f;
    for (int s = 0; s < kRing; s++) lring[(size_t)s * A.plane + o] = 0.f;
  }
}

// ---------------------------------------------------------------------------
// Density transfers transposed (one thread per coarse node of the patch):
// injection (coarse nodes strictly inside took the fine value) and the
// patch boundary nodes (copy at coincident fine nodes, mean of the two
// coarse neighbours at mid nodes).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_adj_inj(AdjInjArgs A) {
  const int a = A.I0 + blockIdx.x * kAT + (threadIdx.x % kAT);
  const int b = A.J0 + blockIdx.y * kAR + (threadIdx.x / kAT);
  if (a > A.I1 || b > A.J1) return;
  const size_t co = at(a, b, A.cpitch);
  const int p = A.pitch, i = 2 * a, j = 2 * b;
  const int L = 2 * A.I0, R = 2 * A.I1, B = 2 * A.J0, T = 2 * A.J1;
  if (a > A.I0 && a < A.I1 && b > A.J0 && b < A.J1) {
    A.lfn[at(i, j, p)] += A.lcn[co];
    A.lcn[co] = 0.f;
    return;
  }
  float s = A.lfn[at(i, j, p)];
  if (b == A.J0 || b == A.J1) {  // horizontal line
    if (i - 1 >= L) s += 0.5f * A.lfn[at(i - 1, j, p)];
    if (i + 1 <= R) s += 0.5f * A.lfn[at(i + 1, j, p)];
  }
  if (a == A.I0 || a == A.I1) {  // vertical line
    if (j - 1 >= B) s += 0.5f * A.lfn[at(i, j - 1, p)];
    if (j + 1 <= T) s += 0.5f * A.lfn[at(i, j + 1, p)];
  }
  A.lcn[co] += s;
}

// ---------------------------------------------------------------------------
// Window close and continuity step (Eq. (4)) transposed, one launch for both
// levels: a block owns a kAdjContTX x kAdjContTY tile of nodes (32 x 5) and
// works over the tile grown by one node.
// Phase 1 (tile + halo): recompute the forward update, clamp mask, ell =
// mask * lam n'; at the own nodes also the E_rms^2 lam into the ring and the
// accumulator (close transposed) and the dF/dA, dF/dbeta partials.  Patch
// boundary nodes took coarse values, so their ell is zero.
// Phase 2 (own nodes): lam n entering the step,
//   lam n_j = ell_j (1 + dt_n nu_j)
//           + c sum_f (ell_j - ell_f) [D'_j (n_f - n_j)/2 - (D_j + D_f)/2],
// c = dt_n/dx^2, over the neighbours f the forward's flux used; written to
// the other lam n buffer (halo reads of lam n leaving never race).
// ---------------------------------------------------------------------------
__device__ inline float d_eff_a(const AdjContArgs& A, float n) {
  if (A.d_const_mode) return A.d_const;
  const float al = n * A.inv_namb;
  return (al * A.Da + A.De) / (1.f + al);
}

__device__ inline float d_eff_prime(const AdjContArgs& A, float n) {
  if (A.d_const_mode) return 0.f;
  const float al = n * A.inv_namb;
  return A.inv_namb * (A.Da - A.De) / ((1.f + al) * (1.f + al));
}

constexpr int kCTX = kAdjContTX, kCTY = kAdjContTY, kCW = kCTX + 2, kCH = kCTY + 2;
constexpr int kCWaves = kAdjContThreads / 64;
static_assert(kCW * kCH <= kAdjContThreads, "one position per thread");

__device__ __forceinline__ void adj_cont_tile(const AdjContArgs& A, int bx, int by,
                                              size_t blk) {
  __shared__ float sEll[kCH][kCW], sN[kCH][kCW];
  __shared__ double sA[kCWaves], sB[kCWaves];
  const int i0 = A.L + bx * kCTX, j0 = A.B + by * kCTY;
  const int tid = threadIdx.x;
  const int p = A.pitch;
  auto cl = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
  double dA = 0.0, dB = 0.0;
  // -- phase 1 --
  if (tid < kCW * kCH) {
    const int ci = tid % kCW, cj = tid / kCW;
    const int i = i0 - 1 + ci, j = j0 - 1 + cj;
    const bool in = i >= A.L && i <= A.R && j >= A.B && j <= A.T;
    const bool own = in && ci >= 1 && ci <= kCTX && cj >= 1 && cj <= kCTY;
    const int ic = cl(i, A.L, A.R), jc = cl(j, A.B, A.T);
    const size_t o = (size_t)jc * p + ic;
    // loads (clamped), then arithmetic
    const float ni = A.n[o], e2 = A.e2[o], lno = A.ln[o];
    const float vl = A.n[(size_t)jc * p + cl(ic - 1, A.L, A.R)];
    const float vr = A.n[(size_t)jc * p + cl(ic + 1, A.L, A.R)];
    const float vd = A.n[(size_t)cl(jc - 1, A.B, A.T) * p + ic];
    const float vu = A.n[(size_t)cl(jc + 1, A.B, A.T) * p + ic];
    const bool edge = A.fine && (i == A.L || i == A.R || j == A.B || j == A.T);
    float lE2 = 0.f, ell = 0.f;
    if (in && !edge) {
      // forward, as the continuity kernel evaluates it
      const float di = d_eff_a(A, ni);
      float flux = 0.f;
      if (i > A.L) flux += 0.5f * (di + d_eff_a(A, vl)) * (vl - ni);
      if (i < A.R) flux += 0.5f * (di + d_eff_a(A, vr)) * (vr - ni);
      if (j > A.B) flux += 0.5f * (di + d_eff_a(A, vd)) * (vd - ni);
      if (j < A.T) flux += 0.5f * (di + d_eff_a(A, vu)) * (vu - ni);
      const float x = e2 * A.eeff_p2;
      // net rate as the continuity kernel evaluates it, and d nu / d E_rms^2
      float nu, pw = 0.f, dnu = 0.f;
      if (A.town) {
        // nu = K y exp(-B / y) - nu_att,  y = sqrt(x) = E_eff / (100 p)
        const float y = sqrtf(x);
        const float ey = y > 0.f ? expf(-A.tB / y) : 0.f;
        nu = (y > 0.f ? A.tK * y * ey : 0.f) - A.tatt;
        if (y > 0.f) dnu = A.tK * ey * (1.f + A.tB / y) * (0.5f * A.eeff_p2 / y);
      } else {
        pw = powf(x, A.half_beta);
        nu = A.nuA * (pw - A.att);
      }
      const float nn = (!A.town && A.rei == 0.f)
                           ? ni + A.dtn * (flux * A.inv_dx2 + nu * ni)
                           : ni + A.dtn * (flux * A.inv_dx2 + (nu - A.rei * ni) * ni);
      // max(0, .): right derivative at 0 (a zero density is perturbed upward)
      ell = nn >= 0.f ? lno : 0.f;
      if (own && A.town) {
        lE2 = ell * A.dtn * ni * dnu;  // A and beta do not enter
      } else if (own) {
        // nu = nu_m A (x^(beta/2) - c^beta),  x = E_rms^2 E_eff-factor/(100 p)^2
        const float lnu = ell * A.dtn * ni;
        if (x > 0.f) {
          lE2 = lnu * A.nuA * A.half_beta * (pw / x) * A.eeff_p2;
          dB = (double)lnu * (double)A.nuA *
               ((double)pw * 0.5 * (double)logf(x) - (double)A.att * (double)A.ln_c);
        } else {
          dB = (double)lnu * (double)A.nuA * (-(double)A.att * (double)A.ln_c);
        }
        dA = (double)lnu * (double)A.nu_m * ((double)pw - (double)A.att);
      }
    }
    sEll[cj][ci] = ell;
    sN[cj][ci] = ni;
    if (own) {
      // close: ring[slot] = acc / spp, acc = 0; E_rms^2 = sum of the ring
      float* rs = A.lring + (size_t)A.slot * A.plane + o;
      const float lsv = *rs + lE2;
      for (int q = 0; q < kRing; q++)
        if (q != A.slot) A.lring[(size_t)q * A.plane + o] += lE2;
      *rs = 0.f;
      A.lacc[o] = lsv * A.inv_spp;
    }
  }
  // block partial sums, fixed order
  for (int d = 32; d >= 1; d >>= 1) {
    dA += __shfl_xor(dA, d, 64);
    dB += __shfl_xor(dB, d, 64);
  }
  const int w = tid >> 6;
  if ((tid & 63) == 0) { sA[w] = dA; sB[w] = dB; }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < kCWaves; k++) { a += sA[k]; b += sB[k]; }
    A.part[2 * blk] = a;
    A.part[2 * blk + 1] = b;
  }
  // -- phase 2 --
  if (tid < kCTX * kCTY) {
    const int tx = tid % kCTX, ty = tid / kCTX;
    const int i = i0 + tx, j = j0 + ty;
    if (i > A.R || j > A.T) return;
    const int ci = tx + 1, cj = ty + 1;
    const size_t o = (size_t)j * p + i;
    const float nj = sN[cj][ci];
    const float dj = d_eff_a(A, nj);
    const float dpj = d_eff_prime(A, nj);
    const float lj = sEll[cj][ci];
    float sacc = 0.f;
    auto face = [&](int a, int b) {
      const float nf = sN[b][a];
      sacc += (lj - sEll[b][a]) * (0.5f * dpj * (nf - nj) - 0.5f * (dj + d_eff_a(A, nf)));
    };
    if (i > A.L) face(ci - 1, cj);
    if (i < A.R) face(ci + 1, cj);
    if (j > A.B) face(ci, cj - 1);
    if (j < A.T) face(ci, cj + 1);
    float self = 0.f;
    if (lj != 0.f) {
      const float x = A.e2[o] * A.eeff_p2;
      float nu;
      if (A.town) {
        const float y = sqrtf(x);
        nu = (y > 0.f ? A.tK * y * expf(-A.tB / y) : 0.f) - A.tatt;
      } else {
        nu = A.nuA * (powf(x, A.half_beta) - A.att);
      }
      // d/dn of n + dtn (nu - r n) n
      self = A.rei == 0.f ? lj * (1.f + A.dtn * nu) : lj * (1.f + A.dtn * (nu - 2.f * A.rei * nj));
    }
    A.ln_o[o] = self + A.dtn * A.inv_dx2 * sacc;
  }
}

// blocks [0, nbf): the patch (F), the rest: the base level (C)
__global__ __launch_bounds__(kAdjContThreads) void k_adj_cont(AdjContArgs F, AdjContArgs C, int nbf,
                                                   int nbfx, int nbcx) {
  const int b = blockIdx.x;
  if (b < nbf) adj_cont_tile(F, b % nbfx, b / nbfx, b);
  else adj_cont_tile(C, (b - nbf) % nbcx, (b - nbf) / nbcx, b);
}

// window close without a continuity step: lam acc = lam ring[slot] / spp
__global__ __launch_bounds__(kThreads) void k_adj_close(AdjContArgs A) {
  const int i = A.L + blockIdx.x * kAT + (threadIdx.x % kAT);
  const int j = A.B + blockIdx.y * kAR + (threadIdx.x / kAT);
  if (i > A.R || j > A.T) return;
  const size_t o = at(i, j, A.pitch);
  float* rs = A.lring + (size_t)A.slot * A.plane + o;
  A.lacc[o] = *rs * A.inv_spp;
  *rs = 0.f;
}

// ---------------------------------------------------------------------------
// Tape plumbing and reductions.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_copy(CopyJobs J) {
  const CopyJob jb = J.job[blockIdx.y];
  const size_t n4 = jb.n / 4;
  const float4* s = reinterpret_cast<const float4*>(jb.src);
  float4* d = reinterpret_cast<float4*>(jb.dst);
  for (size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x; k < n4;
       k += (size_t)gridDim.x * kThreads)
    d[k] = s[k];
}

// sum of the 8 window slots in the order the continuity step adds them
__global__ __launch_bounds__(kThreads) void k_ring_e2(const float* ring, size_t plane,
                                                      int pitch, int L, int B, int R, int T,
                                                      float* dst) {
  const int i = L + blockIdx.x * kAT + (threadIdx.x % kAT);
  const int j = B + blockIdx.y * kAR + (threadIdx.x / kAT);
  if (i > R || j > T) return;
  const size_t o = at(i, j, pitch);
  float e2 = 0.f;
  for (int s = 0; s < kRing; s++) e2 += ring[(size_t)s * plane + o];
  dst[o] = e2;
}

__device__ inline double block_sum(double v, double* sh) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); k++) t += sh[k];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(1024) void k_adj_reduce(const float* src, int nsteps,
                                                     int step_pitch, int rows,
                                                     const double* u, const double* part,
                                                     int nparts, double* out) {
  __shared__ double sh[16];
  // every (step, row) pair of the segment at once: a thread's loads do not
  // wait on one another (a loop over steps would be one memory round trip
  // per step)
  double e0 = 0.0;
  const int n = nsteps * rows;
#pragma unroll 8
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int k = t / rows, q = t - k * rows;
    const float* se = src + (size_t)k * step_pitch;
    e0 += u[2 * k] * (double)se[q] + u[2 * k + 1] * (double)se[rows + q];
  }
  double pa = 0.0, pb = 0.0;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) {
    pa += part[2 * q];
    pb += part[2 * q + 1];
  }
  e0 = block_sum(e0, sh);
  pa = block_sum(pa, sh);
  pb = block_sum(pb, sh);
  if (threadIdx.x == 0) {
    out[0] += e0;
    out[1] += pa;
    out[2] += pb;
  }
}

__global__ __launch_bounds__(kThreads) void k_wdot_part(const float* w, const float* a,
                                                        int pitch, int i0, int j0, int cols,
                                                        int rows, double* part) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  const size_t n = (size_t)cols * rows;
  for (size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (size_t)gridDim.x * kThreads) {
    const int c = (int)(k % cols), r = (int)(k / cols);
    v += (double)w[k] * (double)a[(size_t)(r + j0) * pitch + i0 + c];
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kThreads) void k_wdot_sum(const double* part, int n, double* out) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += kThreads) v += part[k];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ void k_copy2d(const float* src, int spitch, int si0, int sj0, float* dst,
                         int dpitch, int di0, int dj0, int cols, int rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= cols || j >= rows) return;
  dst[(size_t)(j + dj0) * dpitch + di0 + i] = src[(size_t)(j + sj0) * spitch + si0 + i];
}

dim3 node_grid(int L, int B, int R, int T) {
  return dim3((unsigned)((R - L + 1 + kAT - 1) / kAT), (unsigned)((T - B + 1 + kAR - 1) / kAR));
}

}  // namespace

template <bool FINE>
__global__ __launch_bounds__(AdjTile<FINE>::NT) void k_adj_em(AdjEMArgs A) {
  adj_em_tile<FINE>(A, blockIdx.x, blockIdx.y);
}

// patch substep 1 (blocks [0, nbf)) and the base level (the rest) of a base
// step: independent (the base level forms substep 1's boundary G itself)
__global__ __launch_bounds__(AdjTile<true>::NT) void k_adj_em_pair(AdjEMArgs F, AdjEMArgs C, int nbf,
                                                      int nbfx, int nbcx) {
  static_assert(AdjTile<true>::NT == AdjTile<false>::NT, "one block shape");
  const int b = blockIdx.x;
  if (b < nbf) adj_em_tile<true>(F, b % nbfx, b / nbfx);
  else adj_em_tile<false>(C, (b - nbf) % nbcx, (b - nbf) / nbcx);
}

hipError_t launch_adj_em_pair(const AdjEMArgs& F, const AdjEMArgs& C, hipStream_t st) {
  using TF = AdjTile<true>;
  using TC = AdjTile<false>;
  const int nbfx = (F.R - F.L + TF::TX) / TF::TX, nbfy = (F.T - F.B + TF::TY) / TF::TY;
  const int nbcx = (C.R - C.L + TC::TX) / TC::TX, nbcy = (C.T - C.B + TC::TY) / TC::TY;
  const int nbf = nbfx * nbfy;
  k_adj_em_pair<<<nbf + nbcx * nbcy, TF::NT, 0, st>>>(F, C, nbf, nbfx, nbcx);
  return hipGetLastError();
}

hipError_t launch_adj_em(const AdjEMArgs& A, hipStream_t st) {
  if (A.fine) {
    using Tl = AdjTile<true>;
    const dim3 g((A.R - A.L + Tl::TX) / Tl::TX, (A.T - A.B + Tl::TY) / Tl::TY);
    k_adj_em<true><<<g, Tl::NT, 0, st>>>(A);
  } else {
    using Tl = AdjTile<false>;
    const dim3 g((A.R - A.L + Tl::TX) / Tl::TX, (A.T - A.B + Tl::TY) / Tl::TY);
    k_adj_em<false><<<g, Tl::NT, 0, st>>>(A);
  }
  return hipGetLastError();
}

hipError_t launch_adj_grow(const AdjGrowArgs& A, hipStream_t st) {
  k_adj_grow<<<node_grid(A.cL, A.cB, A.cR, A.cT), kThreads, 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_adj_grow_clear(const AdjGrowArgs& A, float* lhz, float* lex, float* ley,
                                 float* ljx, float* ljy, float* ln, float* lacc,
                                 float* lring, hipStream_t st) {
  k_adj_grow_clear<<<node_grid(A.L, A.B, A.R, A.T), kThreads, 0, st>>>(A, lhz, lex, ley, ljx,
                                                                         ljy, ln, lacc, lring);
  return hipGetLastError();
}

hipError_t launch_adj_inj(const AdjInjArgs& A, hipStream_t st) {
  k_adj_inj<<<node_grid(A.I0, A.J0, A.I1, A.J1), kThreads, 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_adj_cont(const AdjContArgs& F, const AdjContArgs& C, int has_f, int* nparts,
                           hipStream_t st) {
  const int nbfx = has_f ? (F.R - F.L + kCTX) / kCTX : 0;
  const int nbf = has_f ? nbfx * ((F.T - F.B + kCTY) / kCTY) : 0;
  const int nbcx = (C.R - C.L + kCTX) / kCTX;
  const int nbc = nbcx * ((C.T - C.B + kCTY) / kCTY);
  k_adj_cont<<<nbf + nbc, kAdjContThreads, 0, st>>>(F, C, nbf, nbfx > 0 ? nbfx : 1, nbcx);
  *nparts = nbf + nbc;
  return hipGetLastError();
}

hipError_t launch_adj_close(const AdjContArgs& A, hipStream_t st) {
  k_adj_close<<<node_grid(A.L, A.B, A.R, A.T), kThreads, 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_copy(const CopyJobs& J, hipStream_t st) {
  if (J.count <= 0) return hipSuccess;
  size_t mx = 0;
  for (int k = 0; k < J.count; k++) mx = J.job[k].n > mx ? J.job[k].n : mx;
  size_t bx = (mx / 4 + kThreads - 1) / kThreads;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  k_copy<<<dim3((unsigned)bx, (unsigned)J.count), kThreads, 0, st>>>(J);
  return hipGetLastError();
}

hipError_t launch_ring_e2(const float* ring, size_t plane, int pitch, int L, int B, int R,
                          int T, float* dst, hipStream_t st) {
  k_ring_e2<<<node_grid(L, B, R, T), kThreads, 0, st>>>(ring, plane, pitch, L, B, R, T, dst);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const float* src, int nsteps, int step_pitch, int rows,
                             const double* u, const double* part, int nparts, double* out,
                             hipStream_t st) {
  k_adj_reduce<<<1, 1024, 0, st>>>(src, nsteps, step_pitch, rows, u, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_copy2d(const float* src, int spitch, int si0, int sj0, float* dst,
                         int dpitch, int di0, int dj0, int cols, int rows, hipStream_t st) {
  if (cols <= 0 || rows <= 0) return hipSuccess;
  k_copy2d<<<dim3((unsigned)((cols + 255) / 256), (unsigned)rows), 256, 0, st>>>(
      src, spitch, si0, sj0, dst, dpitch, di0, dj0, cols, rows);
  return hipGetLastError();
}

hipError_t launch_wdot(const float* w, const float* a, int pitch, int i0, int j0, int cols,
                       int rows, double* part, double* out, hipStream_t st) {
  const size_t n = (size_t)cols * rows;
  int nb = (int)((n + kThreads - 1) / kThreads);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  k_wdot_part<<<nb, kThreads, 0, st>>>(w, a, pitch, i0, j0, cols, rows, part);
  k_wdot_sum<<<1, kThreads, 0, st>>>(part, nb, out);
  return hipGetLastError();
}

}  // namespace dmr
