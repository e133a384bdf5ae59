// dmr_kernels.hip -- gfx950 kernels of the DMR EM / plasma-fluid update.
//
// All kernels work on SoA float32 arrays laid out row-major on the node grid
// of their level: element (i, j) of any entity sits at j*pitch + i, pitch a
// multiple of 64 floats, so one 64-lane wavefront reads one 256-byte row
// segment.  Hz uses cells (i<NX, j<NY), Ex edges (i<NX, j<=NY), Ey edges
// (i<=NX, j<NY), density/window nodes (i<=NX, j<=NY).  The fine level uses
// the same layout on the full-domain fine grid, so the patch can grow without
// moving data; only the patch region is ever touched.
//
// Scaled variables (chosen so the vacuum Yee coefficients are exact in
// float32 at S = 1/2):  H~ = eta0 Hz,  J~ = (dt/eps0) J, with dt the step of
// the level.  Then, per Eqs. (1)-(3):
//   H~ -= S [(Ey_{i+1}-Ey_i) - (Ex_{j+1}-Ex_j)]
//   E+ = [(1-k) E + S dH~ - (1+a)/2 J~] / (1+k),   k = kn n_e
//   J~+ = a J~ + 2k (E + E+)
// E, J, Hz are ping-ponged (read buffer 0, write buffer 1) so a tile can
// recompute its halo without racing its neighbours; the window accumulator
// is updated in place by the tile owning the node.
#include "dmr_kernels.h"

namespace dmr {

// Base-level per-entity arithmetic, shared by the streaming kernel and the
// patch tiles of the combined step (which recompute coarse E on the patch
// boundary lines), so both round identically.
__device__ inline float base_kap(float kn, float n0, float n1) { return kn * (0.5f * (n0 + n1)); }
__device__ inline float base_hz(float hz, float S, float ey1, float ey, float exu, float ex) {
  return hz - S * ((ey1 - ey) - (exu - ex));
}
__device__ inline float base_ex(float e, float kap, float S, float h, float hp, float c1, float j) {
  return ((1.f - kap) * e + S * (h - hp) - c1 * j) * __builtin_amdgcn_rcpf(1.f + kap);
}
__device__ inline float base_ey(float e, float kap, float curl, float c1, float j) {
  return ((1.f - kap) * e + curl - c1 * j) * __builtin_amdgcn_rcpf(1.f + kap);
}

// ---------------------------------------------------------------------------
// Per-entity arithmetic of the patch substep, shared by the one-substep and
// the two-substep kernels so that both round identically.
// ---------------------------------------------------------------------------
// 5-point Laplacian; neighbours outside the patch already replaced by c
__device__ inline float lap5(float c, float l, float r, float d, float u) {
  return l + r + d + u - 4.f * c;
}
// E filter of the patch interior: E - gamma L(L(E))
__device__ inline float filter_e(float e, float gamma, float l2) { return e - gamma * l2; }
// Faraday, Eq. (2), scaled: H~ - S [(Ey_{i+1}-Ey_i) - (Ex_{j+1}-Ex_j)]
__device__ inline float faraday(float ho, float S, float dey, float dex) {
  return ho - S * (dey - dex);
}
// Ampere + Drude, Eqs. (1), (3): new E from the old E, the curl term and J~
// (times the hardware reciprocal of 1 + kap, as the base level: two
// instructions where a correctly rounded division takes eleven)
__device__ inline float ampere(float e, float kap, float curl, float c1, float jo) {
  return ((1.f - kap) * e + curl - c1 * jo) * __builtin_amdgcn_rcpf(1.f + kap);
}
// new J~ = a J~ + 2k (E + E+)
__device__ inline float drude(float a, float jo, float kap, float e, float en) {
  return a * jo + 2.f * kap * (e + en);
}
// Eq. (5b): space weights w0, w1 on two coarse edges, time fraction frac
__device__ inline float cfb(float w0, float w1, float o0, float o1, float n0, float n1,
                            float frac) {
  const float vo = w0 * o0 + w1 * o1;
  const float vn = w0 * n0 + w1 * n1;
  return (1.f - frac) * vo + frac * vn;
}
// window increment of a node from its existing edges (mean per axis)
__device__ inline float win_e2(float sx, int cx, float sy, int cy) {
  return (cx == 2 ? 0.5f * sx : sx) + (cy == 2 ? 0.5f * sy : sy);
}

// ---------------------------------------------------------------------------
// EM substep of the fine patch (Eqs. (1)-(3)), one TX x TY tile of nodes per
// block.  The tile owns Hz(i,j), Ex(i,j), Ey(i,j) and node (i,j) for (i,j)
// in the tile.  It needs old E over [i0-2, i0+TX] x [j0-2, j0+TY] (after the
// patch's E filter, which reads raw E two further out), computes new Hz over
// [i0-2, i0+TX) x [j0-2, j0+TY) and new E over [i0-1, i0+TX) x
// [j0-1, j0+TY) (the halo feeds the node window), then the nodes' E^2.
// Tangential E on the patch boundary comes from the coarse mesh by Eq. (5b);
// with restrict_on, the tile also writes the fine -> coarse transfer of the
// coarse entities strictly inside the patch.
//
// Every global value the tile reads is requested in one batch at the start
// (registers), so the block waits for memory once; the phases after that
// run from LDS and registers.
// ---------------------------------------------------------------------------
// tix: the tile's index in the union's tile list (its slot of the Eq. (5b)
// hand-off between the substeps); unused for the rectangle
// A patch tile's fine arrays from a per-tile corner (ib, jb): entity (i, j)
// at byte offset 4 ((j - jb) pitch + i - ib) of each base.  The offsets stay
// far below 2^32 (a few dozen rows), so loads and stores take a 32-bit
// offset from a uniform base (no per-lane 64-bit address arithmetic);
// pitch * 4 < 2^24 is required by the parameter checks.
struct TileBase {
  const float *hz0, *ex0, *ey0, *jx0, *jy0, *n;
  float *hz1, *ex1, *ey1, *jx1, *jy1, *acc;
  int ib, jb;
  unsigned p4;
  __device__ __forceinline__ TileBase(const EMArgs& A, int ib_, int jb_) : ib(ib_), jb(jb_) {
    const size_t t = (size_t)jb_ * A.pitch + ib_;
    hz0 = A.hz0 + t; ex0 = A.ex0 + t; ey0 = A.ey0 + t;
    jx0 = A.jx0 + t; jy0 = A.jy0 + t; n = A.n + t;
    hz1 = A.hz1 + t; ex1 = A.ex1 + t; ey1 = A.ey1 + t;
    jx1 = A.jx1 + t; jy1 = A.jy1 + t; acc = A.acc + t;
    p4 = (unsigned)A.pitch * 4u;
  }
  __device__ __forceinline__ unsigned off(int i, int j) const {
    return (unsigned)__umul24((unsigned)(j - jb), p4) + ((unsigned)(i - ib) << 2);
  }
};
__device__ __forceinline__ float ldo(const float* p, unsigned b) {
  return *(const float*)((const char*)p + b);
}
__device__ __forceinline__ void sto(float* p, unsigned b, float v) {
  *(float*)((char*)p + b) = v;
}

// LDS of one patch-substep tile (64 x TY nodes), declared by the kernel so
// that the boundary and the interior forms of the tile share it
template <int TY, bool UN>
struct FineLds {
  static constexpr int EW = kTX + 3, EH = TY + 3;  // old E (filtered)
  static constexpr int HW = kTX + 2, HH = TY + 2;  // new Hz
  static constexpr int NW = kTX + 1, NH = TY + 1;  // new E
  static constexpr int DW = kTX + 2, DH = TY + 2;  // density
  static constexpr int RW = kTX + 7, RH = TY + 7;  // raw E for the filter
  static constexpr int QW = kTX + 5, QH = TY + 5;  // Laplacian of raw E
  // Eq. (5b) values: Ex rows B, T; Ey columns L, R.  Union of blocks: Ey on
  // up to 4 block columns (rows 0-3), Ex on up to 2 block rows (4-5)
  static constexpr int NBL = UN ? 6 : 4;
  // union of blocks: activity of the cells [i0-5, i0+kTX+3) x [j0-5, j0+TY+3)
  static constexpr int CW = kTX + 8, CH = TY + 8;
  float rEx[RH][RW], rEy[RH][RW];
  float qEx[QH][QW], qEy[QH][QW];
  float sExo[EH][EW], sEyo[EH][EW];
  float sH[HH][HW], sHo[HH][HW];
  float sExn[NH][NW], sEyn[NH][NW];
  float sN[DH][DW];
  float sJx[TY][kTX], sJy[TY][kTX];
  float sB[NBL + 1][NW > NH ? NW : NH];
  uint8_t sC[UN ? CH : 1][UN ? CW : 1];
};

// A tile whose every entity (raw-E halo included) lies inside the patch
// rectangle and off its boundary lines: no neighbour is replaced, no
// Eq. (5b) value is used, no address needs clamping.
__device__ __forceinline__ bool fine_interior(const EMArgs& A, int i0, int j0, int ty) {
  return i0 - 4 >= A.L && i0 + kTX + 3 <= A.R && j0 - 4 >= A.B && j0 + ty + 3 <= A.T;
}

// IN: the tile is interior (fine_interior); the entity tests below are then
// constant and fold away, with every value computed by the same operations.
template <int TY, int NT, bool UN = false, bool IN = false>
__device__ __forceinline__ void fine_tile(const EMArgs& A, FineLds<TY, UN>& S, int bx, int by,
                                          int tix = 0) {
  static_assert(!(UN && IN), "the interior form is for the patch rectangle");
  using FL = FineLds<TY, UN>;
  constexpr int EW = FL::EW, EH = FL::EH, HW = FL::HW, HH = FL::HH, NW = FL::NW, NH = FL::NH;
  constexpr int DW = FL::DW, DH = FL::DH, RW = FL::RW, RH = FL::RH, QW = FL::QW, QH = FL::QH;
  constexpr int NR = (RH * RW + NT - 1) / NT;
  constexpr int NO = (EH * EW + NT - 1) / NT;
  constexpr int ND = (DH * DW + NT - 1) / NT;
  constexpr int NHZ = (HH * HW + NT - 1) / NT;
  constexpr int NE = (NH * NW + NT - 1) / NT;
  constexpr int RP = NT / kTX;  // tile rows per pass of the block
  constexpr int NA = (TY + RP - 1) / RP;
  constexpr int NBL = FL::NBL, CW = FL::CW, CH = FL::CH;
  auto& rEx = S.rEx; auto& rEy = S.rEy;
  auto& qEx = S.qEx; auto& qEy = S.qEy;
  auto& sExo = S.sExo; auto& sEyo = S.sEyo;
  auto& sH = S.sH; auto& sHo = S.sHo;
  auto& sExn = S.sExn; auto& sEyn = S.sEyn;
  auto& sN = S.sN;
  auto& sJx = S.sJx; auto& sJy = S.sJy;
  auto& sB = S.sB;
  auto& sC = S.sC;

  const int i0 = A.L + bx * kTX;
  const int j0 = A.B + by * TY;
  const int tid = threadIdx.x;
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const int pitch = A.pitch;
  const bool filt = A.gamma > 0.f;
  // which entities belong to the fine level: the patch rectangle, or (union
  // of blocks) a cell in an active block, an edge beside such a cell, a node
  // at one.  ex_in / ey_in (for an edge that belongs): both cells beside it
  // do (else it lies on the coarse/fine boundary).
  auto cact = [&](int i, int j) -> bool { return sC[UN ? j - j0 + 5 : 0][UN ? i - i0 + 5 : 0]; };
  auto hz_ok = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j);
    else if constexpr (IN) return true;
    else return i >= L && i < R && j >= B && j < T;
  };
  auto ex_ok = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j) || cact(i, j - 1);
    else if constexpr (IN) return true;
    else return i >= L && i < R && j >= B && j <= T;
  };
  auto ey_ok = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j) || cact(i - 1, j);
    else if constexpr (IN) return true;
    else return i >= L && i <= R && j >= B && j < T;
  };
  auto nd_ok = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j) || cact(i - 1, j) || cact(i, j - 1) || cact(i - 1, j - 1);
    else if constexpr (IN) return true;
    else return i >= L && i <= R && j >= B && j <= T;
  };
  auto ex_in = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j) && cact(i, j - 1);
    else if constexpr (IN) return true;
    else return j != B && j != T;
  };
  auto ey_in = [&](int i, int j) -> bool {
    if constexpr (UN) return cact(i, j) && cact(i - 1, j);
    else if constexpr (IN) return true;
    else return i != L && i != R;
  };
  // clamped (always valid) addresses of each entity kind
  // (tile-relative byte offsets from the corner (ib, jb), as in fine2_tile)
  const int ib = max(i0 - 8, L), jb = max(j0 - 8, B);
  const TileBase tb(A, ib, jb);
  auto cl = [&](int v, int lo, int hi) {
    if constexpr (IN) return v;
    else return min(max(v, lo), hi);
  };
  auto ob = [&](int i, int j) { return tb.off(i, j); };
  auto o_hz = [&](int i, int j) { return ob(cl(i, L, R - 1), cl(j, B, T - 1)); };
  auto o_ex = [&](int i, int j) { return ob(cl(i, L, R - 1), cl(j, B, T)); };
  auto o_ey = [&](int i, int j) { return ob(cl(i, L, R), cl(j, B, T - 1)); };
  auto o_nd = [&](int i, int j) { return ob(cl(i, L, R), cl(j, B, T)); };

  // -- one batch of global loads ------------------------------------------------
  constexpr int NP = NR > NO ? NR : NO;
  float pex[NP], pey[NP];
  if (filt) {
#pragma unroll
    for (int q = 0; q < NR; q++) {
      const int k = min(tid + q * NT, RH * RW - 1);
      const int i = i0 - 4 + k % RW, j = j0 - 4 + k / RW;
      pex[q] = ldo(tb.ex0, o_ex(i, j));
      pey[q] = ldo(tb.ey0, o_ey(i, j));
    }
  } else {
#pragma unroll
    for (int q = 0; q < NO; q++) {
      const int k = min(tid + q * NT, EH * EW - 1);
      const int i = i0 - 2 + k % EW, j = j0 - 2 + k / EW;
      pex[q] = ldo(tb.ex0, o_ex(i, j));
      pey[q] = ldo(tb.ey0, o_ey(i, j));
    }
  }
  float pn[ND];
#pragma unroll
  for (int q = 0; q < ND; q++) {
    const int k = min(tid + q * NT, DH * DW - 1);
    pn[q] = ldo(tb.n, o_nd(i0 - 1 + k % DW, j0 - 1 + k / DW));
  }
  float phz[NHZ];
#pragma unroll
  for (int q = 0; q < NHZ; q++) {
    const int k = min(tid + q * NT, HH * HW - 1);
    phz[q] = ldo(tb.hz0, o_hz(i0 - 2 + k % HW, j0 - 2 + k / HW));
  }
  float pjx[NE], pjy[NE];
#pragma unroll
  for (int q = 0; q < NE; q++) {
    const int k = min(tid + q * NT, NH * NW - 1);
    const int i = i0 - 1 + k % NW, j = j0 - 1 + k / NW;
    pjx[q] = ldo(tb.jx0, o_ex(i, j));
    pjy[q] = ldo(tb.jy0, o_ey(i, j));
  }
  const int tx = tid % kTX, ty = tid / kTX;
  float pacc[NA];
#pragma unroll
  for (int q = 0; q < NA; q++) pacc[q] = ldo(tb.acc, o_nd(i0 + tx, j0 + ty + q * RP));
  // Eq. (5b) boundary values: x-edges of rows B and T, y-edges of columns L
  // and R inside this tile's new-E region, linear in space between the two
  // nearest coarse edges (weights w0, w1) and in time between the old and
  // new coarse E.  Loads are unconditional (address 0 where unused).
  int bg = -1, bc = 0;
  if constexpr (UN) {
    if (tid < 4 * NH) { bg = tid / NH; bc = tid % NH; }
    else if (tid < 4 * NH + 2 * NW) { bg = 4 + (tid - 4 * NH) / NW; bc = (tid - 4 * NH) % NW; }
  } else if constexpr (!IN) {
    if (tid < NW) { bg = 0; bc = tid; }
    else if (tid < 2 * NW) { bg = 1; bc = tid - NW; }
    else if (tid < 2 * NW + NH) { bg = 2; bc = tid - 2 * NW; }
    else if (tid < 2 * NW + 2 * NH) { bg = 3; bc = tid - 2 * NW - NH; }
  }
  size_t bco = 0, bco2 = 0;
  float bw0 = 0.f, bw1 = 0.f;
  bool bvalid = false;
  // fine edge q of the line at coarse position (q + 1/2)/r - 1/2 between
  // coarse edges c and c + 1 (offsets 1/(2r), Fig. 5(c))
  auto cfb_w = [&](int q, int& c) {
    if (A.rf == 4) {
      const int m = q & 3;
      c = (q >> 2) - (m < 2 ? 1 : 0);
      bw0 = m == 0 ? 0.375f : m == 1 ? 0.125f : m == 2 ? 0.875f : 0.625f;
      bw1 = 1.f - bw0;
    } else if ((q & 1) == 0) {
      c = (q >> 1) - 1; bw0 = 0.25f; bw1 = 0.75f;
    } else {
      c = q >> 1; bw0 = 0.75f; bw1 = 0.25f;
    }
  };
  const int rsh = A.rf == 4 ? 2 : 1;  // fine -> coarse index on a line
  // union of blocks: the block lines crossing the new-E region [i0-1,
  // i0+kTX) x [j0-1, j0+TY), the first at or after i0-1 (j0-1); every
  // position on them gets its Eq. (5b) value, loads clamped into the coarse
  // grid (used only where the edge is on the coarse/fine boundary)
  const int FB = UN ? 1 << A.fbs : 1;
  const int lc0 = UN ? ((i0 - 1 + FB) >> A.fbs << A.fbs) - (((i0 - 1) & (FB - 1)) == 0 ? FB : 0) : 0;
  const int lr0 = UN ? ((j0 - 1 + FB) >> A.fbs << A.fbs) - (((j0 - 1) & (FB - 1)) == 0 ? FB : 0) : 0;
  uint8_t pc[UN ? (CH * CW + NT - 1) / NT : 1];
  if constexpr (UN) {
#pragma unroll
    for (int q = 0; q < (CH * CW + NT - 1) / NT; q++) {
      const int k = min(tid + q * NT, CH * CW - 1);
      const int i = i0 - 5 + k % CW, j = j0 - 5 + k / CW;
      const int bi = i >> A.fbs, bj = j >> A.fbs;  // arithmetic shift: -1 outside
      const bool in = i >= 0 && j >= 0 && bi < A.nbkx && bj < A.nbky;
      pc[q] = A.act[in ? (size_t)bj * A.nbkx + bi : 0];
      if (!in) pc[q] = 0;
    }
    if (bg >= 0 && bg < 4) {  // Ey on a block column
      const int i = lc0 + bg * FB, j = j0 - 1 + bc;
      if (i < i0 + kTX) {
        const int I = min(max(i >> rsh, 0), A.cnx);
        int jc;
        cfb_w(j, jc);
        jc = min(max(jc, 0), A.cny - 2);
        bco = (size_t)jc * A.cpitch + I;
        bco2 = bco + A.cpitch;
        bvalid = true;
      }
    } else if (bg >= 4) {  // Ex on a block row
      const int j = lr0 + (bg - 4) * FB, i = i0 - 1 + bc;
      if (j < j0 + TY) {
        const int J = min(max(j >> rsh, 0), A.cny);
        int ic;
        cfb_w(i, ic);
        ic = min(max(ic, 0), A.cnx - 2);
        bco = (size_t)J * A.cpitch + ic;
        bco2 = bco + 1;
        bvalid = true;
      }
    }
  } else if (bg == 0 || bg == 1) {
    const int i = i0 - 1 + bc, j = bg == 0 ? B : T;
    if (ex_ok(i, j) && j >= j0 - 1 && j < j0 + TY) {
      const int J = j >> rsh;
      int ic;
      cfb_w(i, ic);
      bco = (size_t)J * A.cpitch + ic;
      bco2 = bco + 1;
      bvalid = true;
    }
  } else if (bg >= 2) {
    const int j = j0 - 1 + bc, i = bg == 2 ? L : R;
    if (ey_ok(i, j) && i >= i0 - 1 && i < i0 + kTX) {
      const int I = i >> rsh;
      int jc;
      cfb_w(j, jc);
      bco = (size_t)jc * A.cpitch + I;
      bco2 = bco + A.cpitch;
      bvalid = true;
    }
  }
  const bool bey = UN ? (bg >= 0 && bg < 4) : bg >= 2;  // Ey (else Ex) line
  const float* bp0 = (const float*)(bey ? (uintptr_t)A.cey0 : (uintptr_t)A.cex0);
  const float* bp1 = (const float*)(bey ? (uintptr_t)A.cey1 : (uintptr_t)A.cex1);
  // union, last substep: the Eq. (5b) values come from substep 1 (cfb_prev),
  // because the in-tile fine -> coarse transfer of this launch overwrites
  // coarse edges next to the boundary at concave corners
  const bool from_prev = UN && A.cfb_prev != nullptr;
  if (from_prev) bco = bco2 = 0;
  float bo0 = 0.f, bo1 = 0.f, bn0 = 0.f, bn1 = 0.f;
  if constexpr (!IN) { bo0 = bp0[bco]; bo1 = bp0[bco2]; bn0 = bp1[bco]; bn1 = bp1[bco2]; }
  float bpre = 0.f;
  if constexpr (UN) {
    if (from_prev && bg >= 0) bpre = A.cfb_prev[(size_t)tix * kCfbStride + tid];
  }

  if constexpr (UN) {
#pragma unroll
    for (int q = 0; q < (CH * CW + NT - 1) / NT; q++) {
      const int k = tid + q * NT;
      if (k < CH * CW) sC[k / CW][k % CW] = pc[q];
    }
    __syncthreads();
  }

  // -- old E: raw, Laplacian, filtered ----------------------------------------
  // Weak fourth-order hyper-diffusion of the patch's interior E before the
  // substep, E <- E - gamma L(L(E)) per component on its own grid, with
  // neighbours outside the patch replaced by the centre value; the
  // coarse-driven boundary edges are left as they are.
  if (filt) {
#pragma unroll
    for (int q = 0; q < NR; q++) {
      const int k = tid + q * NT;
      if (k < RH * RW) {
        const int ci = k % RW, cj = k / RW;
        const int i = i0 - 4 + ci, j = j0 - 4 + cj;
        rEx[cj][ci] = ex_ok(i, j) ? pex[q] : 0.f;
        rEy[cj][ci] = ey_ok(i, j) ? pey[q] : 0.f;
      }
    }
    __syncthreads();
    for (int k = tid; k < QH * QW; k += NT) {
      const int ci = k % QW, cj = k / QW;
      const int i = i0 - 3 + ci, j = j0 - 3 + cj;
      const int a = ci + 1, b = cj + 1;  // raw coordinates
      float lx = 0.f, ly = 0.f;
      if (ex_ok(i, j)) {
        const float c = rEx[b][a];
        lx = lap5(c, ex_ok(i - 1, j) ? rEx[b][a - 1] : c, ex_ok(i + 1, j) ? rEx[b][a + 1] : c,
                  ex_ok(i, j - 1) ? rEx[b - 1][a] : c, ex_ok(i, j + 1) ? rEx[b + 1][a] : c);
      }
      if (ey_ok(i, j)) {
        const float c = rEy[b][a];
        ly = lap5(c, ey_ok(i - 1, j) ? rEy[b][a - 1] : c, ey_ok(i + 1, j) ? rEy[b][a + 1] : c,
                  ey_ok(i, j - 1) ? rEy[b - 1][a] : c, ey_ok(i, j + 1) ? rEy[b + 1][a] : c);
      }
      qEx[cj][ci] = lx;
      qEy[cj][ci] = ly;
    }
    __syncthreads();
    for (int k = tid; k < EH * EW; k += NT) {
      const int ci = k % EW, cj = k / EW;
      const int i = i0 - 2 + ci, j = j0 - 2 + cj;
      const int a = ci + 1, b = cj + 1;  // Laplacian coordinates
      float ex = 0.f, ey = 0.f;
      if (ex_ok(i, j)) {
        ex = rEx[cj + 2][ci + 2];
        if (ex_in(i, j)) {
          const float c = qEx[b][a];
          const float l2 = lap5(c, ex_ok(i - 1, j) ? qEx[b][a - 1] : c, ex_ok(i + 1, j) ? qEx[b][a + 1] : c,
                                ex_ok(i, j - 1) ? qEx[b - 1][a] : c, ex_ok(i, j + 1) ? qEx[b + 1][a] : c);
          ex = filter_e(ex, A.gamma, l2);
        }
      }
      if (ey_ok(i, j)) {
        ey = rEy[cj + 2][ci + 2];
        if (ey_in(i, j)) {
          const float c = qEy[b][a];
          const float l2 = lap5(c, ey_ok(i - 1, j) ? qEy[b][a - 1] : c, ey_ok(i + 1, j) ? qEy[b][a + 1] : c,
                                ey_ok(i, j - 1) ? qEy[b - 1][a] : c, ey_ok(i, j + 1) ? qEy[b + 1][a] : c);
          ey = filter_e(ey, A.gamma, l2);
        }
      }
      sExo[cj][ci] = ex;
      sEyo[cj][ci] = ey;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NO; q++) {
      const int k = tid + q * NT;
      if (k < EH * EW) {
        const int ci = k % EW, cj = k / EW;
        const int i = i0 - 2 + ci, j = j0 - 2 + cj;
        sExo[cj][ci] = ex_ok(i, j) ? pex[q] : 0.f;
        sEyo[cj][ci] = ey_ok(i, j) ? pey[q] : 0.f;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < ND; q++) {
    const int k = tid + q * NT;
    if (k < DH * DW) {
      const int ci = k % DW, cj = k / DW;
      sN[cj][ci] = nd_ok(i0 - 1 + ci, j0 - 1 + cj) ? pn[q] : 0.f;
    }
  }
  if constexpr (!IN) {  // every thread writes (row NBL is a dummy), so the loads above stay put
    sB[bg < 0 ? NBL : bg][bg < 0 ? 0 : bc] =
        from_prev ? bpre : (bvalid ? cfb(bw0, bw1, bo0, bo1, bn0, bn1, A.frac) : 0.f);
    if constexpr (UN) {  // substep 1 hands the last substep its values (frac = 1)
      if (A.cfb_next && bg >= 0)
        A.cfb_next[(size_t)tix * kCfbStride + tid] =
            bvalid ? cfb(bw0, bw1, bo0, bo1, bn0, bn1, 1.f) : 0.f;
    }
  }
  __syncthreads();

  // -- Faraday, Eq. (2) -------------------------------------------------------
#pragma unroll
  for (int q = 0; q < NHZ; q++) {
    const int k = tid + q * NT;
    if (k < HH * HW) {
      const int ci = k % HW, cj = k / HW;
      const int i = i0 - 2 + ci, j = j0 - 2 + cj;
      float h = 0.f, ho = 0.f;
      if (hz_ok(i, j)) {
        const unsigned o = ob(i, j);
        const float dey = sEyo[cj][ci + 1] - sEyo[cj][ci];
        const float dex = sExo[cj + 1][ci] - sExo[cj][ci];
        ho = phz[q];
        h = faraday(ho, A.S, dey, dex);
        if (ci >= 2 && cj >= 2) {
          sto(tb.hz1, o, h);
          if (A.hz_save) A.hz_save[(size_t)j * pitch + i] = h;
        }
      }
      sH[cj][ci] = h;
      sHo[cj][ci] = ho;
    }
  }
  __syncthreads();

  // -- Ampere + Drude, Eqs. (1), (3); Eq. (5b) on the boundary ------------------
#pragma unroll
  for (int q = 0; q < NE; q++) {
    const int k = tid + q * NT;
    if (k < NH * NW) {
      const int ci = k % NW, cj = k / NW;
      const int i = i0 - 1 + ci, j = j0 - 1 + cj;
      const bool own = ci >= 1 && cj >= 1;
      const unsigned o = ob(i, j);
      float exn = 0.f, eyn = 0.f;
      if (ex_ok(i, j)) {
        const float e = sExo[cj + 1][ci + 1];
        const float ne = 0.5f * (sN[cj][ci] + sN[cj][ci + 1]);
        const float kap = A.kn * ne;
        const float jo = pjx[q];
        if (ex_in(i, j)) {
          const float dh = sH[cj + 1][ci + 1] - sH[cj][ci + 1];
          exn = ampere(e, kap, A.S * dh, A.c1, jo);
        } else if constexpr (UN) {
          exn = sB[4 + ((j - lr0) >> A.fbs)][ci];
        } else {
          exn = sB[j == B ? 0 : 1][ci];
        }
        if (own) {
          const float jn = drude(A.a, jo, kap, e, exn);
          sto(tb.ex1, o, exn);
          sto(tb.jx1, o, jn);
          sJx[cj - 1][ci - 1] = jn;
        }
      }
      if (ey_ok(i, j)) {
        const float e = sEyo[cj + 1][ci + 1];
        const float ne = 0.5f * (sN[cj][ci] + sN[cj + 1][ci]);
        const float kap = A.kn * ne;
        const float jo = pjy[q];
        if (ey_in(i, j)) {
          const float dh = sH[cj + 1][ci + 1] - sH[cj + 1][ci];
          eyn = ampere(e, kap, -A.S * dh, A.c1, jo);
        } else if constexpr (UN) {
          eyn = sB[(i - lc0) >> A.fbs][cj];
        } else {
          eyn = sB[i == L ? 2 : 3][cj];
        }
        if (own) {
          const float jn = drude(A.a, jo, kap, e, eyn);
          sto(tb.ey1, o, eyn);
          sto(tb.jy1, o, jn);
          sJy[cj - 1][ci - 1] = jn;
        }
      }
      sExn[cj][ci] = exn;
      sEyn[cj][ci] = eyn;
    }
  }
  __syncthreads();

  // -- window accumulation at the tile's nodes ---------------------------------
#pragma unroll
  for (int q = 0; q < NA; q++) {
    const int r = ty + q * RP;
    const int i = i0 + tx, j = j0 + r;
    if (r >= TY || !nd_ok(i, j)) continue;
    const int ci = tx + 1, cj = r + 1;
    float sx = 0.f, sy = 0.f;
    int cx = 0, cy = 0;
    // the node's own edges (rectangle: i > L is Ex(i-1, j) belonging, ...)
    const bool xl = IN || (UN ? ex_ok(i - 1, j) : i > L), xr = IN || (UN ? ex_ok(i, j) : i < R);
    const bool yd = IN || (UN ? ey_ok(i, j - 1) : j > B), yu = IN || (UN ? ey_ok(i, j) : j < T);
    if (xl) { const float v = sExn[cj][ci - 1]; sx += v * v; cx++; }
    if (xr) { const float v = sExn[cj][ci]; sx += v * v; cx++; }
    if (yd) { const float v = sEyn[cj - 1][ci]; sy += v * v; cy++; }
    if (yu) { const float v = sEyn[cj][ci]; sy += v * v; cy++; }
    const float e2 = win_e2(sx, cx, sy, cy);
    sto(tb.acc, ob(i, j), pacc[q] + e2);
  }

  // -- fine -> coarse transfer after the last substep ------------------------
  if (A.restrict_on && A.rf != 4) {
    for (int r = ty; r < TY; r += RP) {
      const int i = i0 + tx, j = j0 + r;
      if (((i - L) | (j - B)) & 1) continue;
      const int a = i >> 1, b = j >> 1;
      const size_t co = (size_t)b * A.cpitch + a;
      const int ci = tx + 1, cj = r + 1;   // new-E coordinates of (i, j)
      if (hz_ok(i, j)) {
        float s = 0.f;
        for (int da = 0; da < 2; da++)
          for (int db = 0; db < 2; db++) {
            const float hold = sHo[r + 2 + db][tx + 2 + da];
            s += 0.5f * (hold + sH[r + 2 + db][tx + 2 + da]);
          }
        A.chz[co] = 0.25f * s;
      }
      if (ex_ok(i, j) && ex_in(i, j)) {
        A.cex[co] = 0.5f * (sExn[cj][ci] + sExn[cj][ci + 1]);
        A.cjx[co] = sJx[r][tx] + sJx[r][tx + 1];  // J~ scales with dt
      }
      if (ey_ok(i, j) && ey_in(i, j)) {
        A.cey[co] = 0.5f * (sEyn[cj][ci] + sEyn[cj + 1][ci]);
        A.cjy[co] = sJy[r][tx] + sJy[r + 1][tx];
      }
    }
  } else if (A.restrict_on) {
    // r = 4: 4 x 4 cells and the half levels after substeps 2 (hz_lo, global)
    // and 3 (the Hz entering this last substep); 4 edges, J~ summed
    for (int r = ty; r < TY; r += RP) {
      const int i = i0 + tx, j = j0 + r;
      if (((i - L) | (j - B)) & 3) continue;
      const int a = i >> 2, b = j >> 2;
      const size_t co = (size_t)b * A.cpitch + a;
      const int ci = tx + 1, cj = r + 1;
      if (hz_ok(i, j)) {
        float s = 0.f;
        for (int da = 0; da < 4; da++)
          for (int db = 0; db < 4; db++) {
            const float lo = A.hz_lo[(size_t)(j + db) * pitch + i + da];
            s += 0.5f * (lo + sHo[r + 2 + db][tx + 2 + da]);
          }
        A.chz[co] = 0.0625f * s;
      }
      if (ex_ok(i, j) && j > B && j < T) {
        float se = 0.f, sj = 0.f;
        for (int da = 0; da < 4; da++) { se += sExn[cj][ci + da]; sj += sJx[r][tx + da]; }
        A.cex[co] = 0.25f * se;
        A.cjx[co] = sj;
      }
      if (ey_ok(i, j) && i > L && i < R) {
        float se = 0.f, sj = 0.f;
        for (int db = 0; db < 4; db++) { se += sEyn[cj + db][ci]; sj += sJy[r + db][tx]; }
        A.cey[co] = 0.25f * se;
        A.cjy[co] = sj;
      }
    }
  }
}

// Two 1024-thread tiles share a CU only if each wave holds at most 80
// scalar registers (more leaves one tile per CU); the interior form would
// otherwise take 88.
template <int TY, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_num_sgpr(kTileSgprs))) void k_fine(EMArgs A) {
  __shared__ FineLds<TY, false> S;
  const int bx = blockIdx.x, by = blockIdx.y;
  if (fine_interior(A, A.L + bx * kTX, A.B + by * TY, TY))
    fine_tile<TY, NT, false, true>(A, S, bx, by);
  else
    fine_tile<TY, NT>(A, S, bx, by);
}

// the fine level as a union of blocks: one listed tile per block
template <int TY, int NT>
__global__ __launch_bounds__(NT) void k_fine_union(EMArgs A, const int2* __restrict__ tiles) {
  __shared__ FineLds<TY, true> S;
  const int2 t = tiles[blockIdx.x];
  fine_tile<TY, NT, true>(A, S, t.x, t.y, blockIdx.x);
}

// batched union levels: blk[b] = (instance, index in the instance's tile list)
template <int TY>
__global__ __launch_bounds__(kFineThreads) void k_fine_union_batch(const EMArgs* __restrict__ args,
                                                                   const int2* __restrict__ blk) {
  const int2 bi = blk[blockIdx.x];
  const EMArgs& A = args[bi.x];
  __shared__ FineLds<TY, true> S;
  const int2 t = A.utiles[bi.y];
  fine_tile<TY, kFineThreads, true>(A, S, t.x, t.y, bi.y);
}

// Eq. (5b) source of thread tid for one substep's new-E region (origin orig
// relative to the tile corner, NW_ x NH_): group g (x-edges of row B / T,
// y-edges of column L / R, -1 none), position c, the two coarse edges o, o2
// (o at coarse column / row cidx along the line) with weights w0, w1;
// ok = the edge exists and lies in the region.  r4: refinement factor 4
// (offsets 1/8: weights 3/8, 1/8, 7/8, 5/8 on the lower coarse edge).
__device__ __forceinline__ void bnd_src(int tid, int orig, int NW_, int NH_, int i0, int j0,
                                        int L, int R, int B, int T, int cpitch, int& g,
                                        int& c, size_t& o, size_t& o2, float& w0, float& w1,
                                        bool& ok, int& cidx, bool r4 = false) {
  // fine edge q of a line: lower coarse edge and its weight
  auto wq = [&](int q, int& cq) {
    if (r4) {
      const int m = q & 3;
      cq = (q >> 2) - (m < 2 ? 1 : 0);
      w0 = m == 0 ? 0.375f : m == 1 ? 0.125f : m == 2 ? 0.875f : 0.625f;
      w1 = 1.f - w0;
    } else if ((q & 1) == 0) {
      cq = (q >> 1) - 1; w0 = 0.25f; w1 = 0.75f;
    } else {
      cq = q >> 1; w0 = 0.75f; w1 = 0.25f;
    }
  };
  const int rsh = r4 ? 2 : 1;
  g = -1; c = 0; o = 0; o2 = 0; w0 = 0.f; w1 = 0.f; ok = false; cidx = 0;
  if (tid < NW_) { g = 0; c = tid; }
  else if (tid < 2 * NW_) { g = 1; c = tid - NW_; }
  else if (tid < 2 * NW_ + NH_) { g = 2; c = tid - 2 * NW_; }
  else if (tid < 2 * NW_ + 2 * NH_) { g = 3; c = tid - 2 * NW_ - NH_; }
  if (g == 0 || g == 1) {
    const int i = i0 + orig + c, j = g == 0 ? B : T;
    if (i >= L && i < R && j >= j0 + orig && j < j0 + orig + NH_) {
      int ic;
      wq(i, ic);
      o = (size_t)(j >> rsh) * cpitch + ic;
      o2 = o + 1;
      ok = true;
      cidx = ic;
    }
  } else if (g >= 2) {
    const int j = j0 + orig + c, i = g == 2 ? L : R;
    if (j >= B && j < T && i >= i0 + orig && i < i0 + orig + NW_) {
      int jc;
      wq(j, jc);
      o = (size_t)jc * cpitch + (i >> rsh);
      o2 = o + cpitch;
      ok = true;
      cidx = jc;
    }
  }
}

// ---------------------------------------------------------------------------
// Both patch substeps of a coarse step in one launch (temporal blocking).
// Substep 1 runs over the tile grown by 3 cells on every side and stays in
// LDS; substep 2 runs over the tile from those values and is the only one
// written (fields, window, fine -> coarse transfer).  Reads the patch state
// from buffer 0 and writes buffer 1.  Each entity is computed with the same
// operations as by the two one-substep launches (the helpers above), so the
// results are identical.  Region origins are relative to the tile corner
// (i0, j0):  raw E0 -7, L(E0) -6, filtered E0 and H1 -5, E1/J1 and n -4;
// then as in fine_tile: L(E1) -3, filtered E1 and H2 -2, E2/J2 -1.
// R4: refinement factor 4, the launch runs substeps (1, 2) or (3, 4) of a
// coarse step (A.frac = time fraction of the first); the fine -> coarse
// transfer (A.restrict_on, second pair) uses the Hz after substep 2, which
// is this launch's input, and after substep 3 (H1).
// ---------------------------------------------------------------------------
template <int TY, int NT, bool LOCAL, bool ST = false, bool R4 = false, int TW = kTX>
__device__ __forceinline__ void fine2_tile(const EMArgs& A, int bx, int by, float cey_src,
                                           float chz_src) {
  constexpr int R1W = TW + 13, R1H = TY + 13;
  constexpr int Q1W = TW + 11, Q1H = TY + 11;
  constexpr int F1W = TW + 9, F1H = TY + 9;
  constexpr int H1W = TW + 8, H1H = TY + 8;
  constexpr int N1W = TW + 7, N1H = TY + 7;
  constexpr int D1W = TW + 8, D1H = TY + 8;
  constexpr int Q2W = TW + 5, Q2H = TY + 5;
  constexpr int F2W = TW + 3, F2H = TY + 3;
  constexpr int H2W = TW + 2, H2H = TY + 2;
  constexpr int N2W = TW + 1, N2H = TY + 1;
  constexpr int NR = (R1H * R1W + NT - 1) / NT;
  constexpr int NH0 = (H1H * H1W + NT - 1) / NT;
  constexpr int NJ0 = (N1H * N1W + NT - 1) / NT;
  constexpr int ND = (D1H * D1W + NT - 1) / NT;
  constexpr int RP = NT / TW;  // tile rows per pass of the block
  constexpr int NA = (TY + RP - 1) / RP;
  __shared__ float rX[R1H][R1W], rY[R1H][R1W];  // raw E0
  __shared__ float qX[Q1H][Q1W], qY[Q1H][Q1W];  // L(E0), then L(E1)
  __shared__ float fX[F1H][F1W], fY[F1H][F1W];  // filtered E0, then filtered E1
  __shared__ float sH1[H1H][H1W];
  __shared__ float e1X[N1H][N1W], e1Y[N1H][N1W];
  __shared__ float j1X[N2H][N2W], j1Y[N2H][N2W];
  __shared__ float sN[D1H][D1W];
  __shared__ float sH2[H2H][H2W];
  __shared__ float e2X[N2H][N2W], e2Y[N2H][N2W];
  __shared__ float j2X[TY][TW], j2Y[TY][TW];
  __shared__ float sB1[5][N1W], sB2[5][N2W];  // Eq. (5b) values of substeps 1 and 2

  const int i0 = A.L + bx * TW;
  const int j0 = A.B + by * TY;
  const int tid = threadIdx.x;
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const int pitch = A.pitch;
  const bool filt = A.gamma > 0.f;
  const float frac1 = A.frac, frac2 = R4 ? A.frac + 0.25f : 1.f;
  auto hz_ok = [=](int i, int j) { return i >= L && i < R && j >= B && j < T; };
  auto ex_ok = [=](int i, int j) { return i >= L && i < R && j >= B && j <= T; };
  auto ey_ok = [=](int i, int j) { return i >= L && i <= R && j >= B && j < T; };
  auto nd_ok = [=](int i, int j) { return i >= L && i <= R && j >= B && j <= T; };
  // tile-relative byte offsets: every fine entity the tile reads or writes
  // lies in [ib, ib + TW + 16) x [jb, jb + TY + 16) (clamped loads
  // included), so a 32-bit offset from per-tile bases addresses it
  const int ib = max(i0 - 8, L), jb = max(j0 - 8, B);
  const TileBase tb(A, ib, jb);
  auto cl = [=](int v, int lo, int hi) { return min(max(v, lo), hi); };
  auto ob = [=](int i, int j) { return tb.off(i, j); };
  auto o_hz = [=](int i, int j) { return ob(cl(i, L, R - 1), cl(j, B, T - 1)); };
  auto o_ex = [=](int i, int j) { return ob(cl(i, L, R - 1), cl(j, B, T)); };
  auto o_ey = [=](int i, int j) { return ob(cl(i, L, R), cl(j, B, T - 1)); };
  auto o_nd = [=](int i, int j) { return ob(cl(i, L, R), cl(j, B, T)); };

  // -- one batch of global loads ------------------------------------------------
  float pex[NR], pey[NR];
#pragma unroll
  for (int q = 0; q < NR; q++) {
    const int k = min(tid + q * NT, R1H * R1W - 1);
    const int i = i0 - 7 + k % R1W, j = j0 - 7 + k / R1W;
    pex[q] = ldo(tb.ex0, o_ex(i, j));
    pey[q] = ldo(tb.ey0, o_ey(i, j));
  }
  float phz[NH0];
#pragma unroll
  for (int q = 0; q < NH0; q++) {
    const int k = min(tid + q * NT, H1H * H1W - 1);
    phz[q] = ldo(tb.hz0, o_hz(i0 - 5 + k % H1W, j0 - 5 + k / H1W));
  }
  float pjx[NJ0], pjy[NJ0];
#pragma unroll
  for (int q = 0; q < NJ0; q++) {
    const int k = min(tid + q * NT, N1H * N1W - 1);
    const int i = i0 - 4 + k % N1W, j = j0 - 4 + k / N1W;
    pjx[q] = ldo(tb.jx0, o_ex(i, j));
    pjy[q] = ldo(tb.jy0, o_ey(i, j));
  }
  float pn[ND];
#pragma unroll
  for (int q = 0; q < ND; q++) {
    const int k = min(tid + q * NT, D1H * D1W - 1);
    pn[q] = ldo(tb.n, o_nd(i0 - 4 + k % D1W, j0 - 4 + k / D1W));
  }
  const int tx = tid % TW, ty = tid / TW;
  float pacc[NA];
#pragma unroll
  for (int q = 0; q < NA; q++) pacc[q] = ldo(tb.acc, o_nd(i0 + tx, j0 + ty + q * RP));
  // Eq. (5b) sources of both substeps: boundary x-edges of rows B, T and
  // y-edges of columns L, R inside each substep's new-E region (origin
  // -4 of width N1W x N1H for substep 1, -1 of N2W x N2H for substep 2)
  int g1, c1_, g2, c2, k1, k2;
  size_t o1a, o1b, o2a, o2b;
  float w1a, w1b, w2a, w2b;
  bool ok1, ok2;
  bnd_src(tid, -4, N1W, N1H, i0, j0, L, R, B, T, A.cpitch, g1, c1_, o1a, o1b, w1a, w1b, ok1, k1, R4);
  bnd_src(tid, -1, N2W, N2H, i0, j0, L, R, B, T, A.cpitch, g2, c2, o2a, o2b, w2a, w2b, ok2, k2, R4);
  // addresses selected as integers (a select of two argument pointers can
  // otherwise be lowered through private memory)
  const float* b1o = (const float*)(g1 >= 2 ? (uintptr_t)A.cey0 : (uintptr_t)A.cex0);
  const float* b2o = (const float*)(g2 >= 2 ? (uintptr_t)A.cey0 : (uintptr_t)A.cex0);
  const float b1v0 = b1o[o1a], b1v1 = b1o[o1b];
  const float b2v0 = b2o[o2a], b2v1 = b2o[o2b];
  float b1v2 = 0.f, b1v3 = 0.f, b2v2 = 0.f, b2v3 = 0.f;
  if constexpr (!LOCAL) {
    const float* b1n = (const float*)(g1 >= 2 ? (uintptr_t)A.cey1 : (uintptr_t)A.cex1);
    const float* b2n = (const float*)(g2 >= 2 ? (uintptr_t)A.cey1 : (uintptr_t)A.cex1);
    b1v2 = b1n[o1a]; b1v3 = b1n[o1b];
    b2v2 = b2n[o2a]; b2v3 = b2n[o2b];
  }
  // combined step: the coarse E after the coarse step on the patch boundary
  // lines is computed here from the coarse state entering it (the base-level
  // waves of the same launch compute the same values).  x-lines: coarse rows
  // B/r and T/r at columns [cx0, cx0 + CW); y-lines: coarse columns L/r and
  // R/r at rows [cy0, cy0 + CH) (enough for r = 2; r = 4 needs fewer).
  constexpr int RS = R4 ? 2 : 1;  // fine -> coarse index shift
  constexpr int CW = TW / 2 + 6, CH = TY / 2 + 6;
  __shared__ float sC[5][CW > CH ? CW : CH];
  const int cx0 = ((i0 - 4) >> RS) - 1, cy0 = ((j0 - 4) >> RS) - 1;
  int cg = -1, cc = 0;
  float q[12];
  if constexpr (LOCAL) {
    if (tid < CW) { cg = 0; cc = tid; }
    else if (tid < 2 * CW) { cg = 1; cc = tid - CW; }
    else if (tid < 2 * CW + CH) { cg = 2; cc = tid - 2 * CW; }
    else if (tid < 2 * CW + 2 * CH) { cg = 3; cc = tid - 2 * CW - CH; }
    const int cp = A.cpitch, NXc = A.cnx, NYc = A.cny;
    auto cidx = [=](int a, int b) {  // clamped coarse address
      const int aa = a < 0 ? 0 : (a > NXc ? NXc : a), bb = b < 0 ? 0 : (b > NYc ? NYc : b);
      return (size_t)bb * cp + aa;
    };
    if (cg <= 1) {  // x-edge (ic, J) of a boundary row (threads without a role: cg = -1)
      const int ic = cx0 + cc, J = cg == 1 ? (T >> RS) : (B >> RS);
      q[0] = A.cex0[cidx(ic, J - 1)]; q[1] = A.cex0[cidx(ic, J)]; q[2] = A.cex0[cidx(ic, J + 1)];
      q[3] = A.cey0[cidx(ic, J - 1)]; q[4] = A.cey0[cidx(ic + 1, J - 1)];
      q[5] = A.cey0[cidx(ic, J)]; q[6] = A.cey0[cidx(ic + 1, J)];
      q[7] = A.chz0[cidx(ic, J - 1)]; q[8] = A.chz0[cidx(ic, J)];
      q[9] = A.cjx0[cidx(ic, J)]; q[10] = A.cn0[cidx(ic, J)]; q[11] = A.cn0[cidx(ic + 1, J)];
    } else {        // y-edge (I, jc) of a boundary column
      const int jc = cy0 + cc, I = cg == 3 ? (R >> RS) : (L >> RS);
      q[0] = A.cey0[cidx(I - 1, jc)]; q[1] = A.cey0[cidx(I, jc)]; q[2] = A.cey0[cidx(I + 1, jc)];
      q[3] = A.cex0[cidx(I - 1, jc)]; q[4] = A.cex0[cidx(I - 1, jc + 1)];
      q[5] = A.cex0[cidx(I, jc)]; q[6] = A.cex0[cidx(I, jc + 1)];
      q[7] = A.chz0[cidx(I - 1, jc)]; q[8] = A.chz0[cidx(I, jc)];
      q[9] = A.cjy0[cidx(I, jc)]; q[10] = A.cn0[cidx(I, jc)]; q[11] = A.cn0[cidx(I, jc + 1)];
    }
  }

  // -- substep 1: raw E0 first (the filter's first phase needs nothing else),
// then n and the boundary values while the Laplacian of E0 is formed, so
// the other loads are still in flight during that phase
#pragma unroll
  for (int q = 0; q < NR; q++) {
    const int k = tid + q * NT;
    if (k < R1H * R1W) {
      const int ci = k % R1W, cj = k / R1W;
      const int i = i0 - 7 + ci, j = j0 - 7 + cj;
      rX[cj][ci] = ex_ok(i, j) ? pex[q] : 0.f;
      rY[cj][ci] = ey_ok(i, j) ? pey[q] : 0.f;
    }
  }
  __syncthreads();
  // filter of E0: L over origin -6, filtered over origin -5
  auto laplace = [&](const float (*rx)[R1W], const float (*ry)[R1W], int rorg, int qorg, int QW,
                     int QH) {
    for (int k = tid; k < QH * QW; k += NT) {
      const int ci = k % QW, cj = k / QW;
      const int i = i0 + qorg + ci, j = j0 + qorg + cj;
      const int a = ci + (qorg - rorg), b = cj + (qorg - rorg);  // raw coordinates
      // all ten reads first (the raw region reaches one entity past this
      // one on every side), then the selects: one LDS round trip
      const float xc = rx[b][a], xl = rx[b][a - 1], xr = rx[b][a + 1], xd = rx[b - 1][a],
                  xu = rx[b + 1][a];
      const float yc = ry[b][a], yl = ry[b][a - 1], yr = ry[b][a + 1], yd = ry[b - 1][a],
                  yu = ry[b + 1][a];
      const float lx = lap5(xc, ex_ok(i - 1, j) ? xl : xc, ex_ok(i + 1, j) ? xr : xc,
                            ex_ok(i, j - 1) ? xd : xc, ex_ok(i, j + 1) ? xu : xc);
      const float ly = lap5(yc, ey_ok(i - 1, j) ? yl : yc, ey_ok(i + 1, j) ? yr : yc,
                            ey_ok(i, j - 1) ? yd : yc, ey_ok(i, j + 1) ? yu : yc);
      qX[cj][ci] = ex_ok(i, j) ? lx : 0.f;
      qY[cj][ci] = ey_ok(i, j) ? ly : 0.f;
    }
  };
  auto filtered = [&](const float (*rx)[R1W], const float (*ry)[R1W], int rorg, int forg, int FW,
                      int FH) {
    for (int k = tid; k < FH * FW; k += NT) {
      const int ci = k % FW, cj = k / FW;
      const int i = i0 + forg + ci, j = j0 + forg + cj;
      const int a = ci + 1, b = cj + 1;                          // Laplacian coordinates
      const int ra = ci + (forg - rorg), rb = cj + (forg - rorg);  // raw coordinates
      // every read first (the Laplacian region reaches one entity past this
      // one; without the filter its values are unused), then the selects
      const float ex = rx[rb][ra], ey = ry[rb][ra];
      const float xc = qX[b][a], xl = qX[b][a - 1], xr = qX[b][a + 1], xd = qX[b - 1][a],
                  xu = qX[b + 1][a];
      const float yc = qY[b][a], yl = qY[b][a - 1], yr = qY[b][a + 1], yd = qY[b - 1][a],
                  yu = qY[b + 1][a];
      const float fx = filter_e(ex, A.gamma,
                                lap5(xc, ex_ok(i - 1, j) ? xl : xc, ex_ok(i + 1, j) ? xr : xc,
                                     ex_ok(i, j - 1) ? xd : xc, ex_ok(i, j + 1) ? xu : xc));
      const float fy = filter_e(ey, A.gamma,
                                lap5(yc, ey_ok(i - 1, j) ? yl : yc, ey_ok(i + 1, j) ? yr : yc,
                                     ey_ok(i, j - 1) ? yd : yc, ey_ok(i, j + 1) ? yu : yc));
      fX[cj][ci] = ex_ok(i, j) ? ((filt && j != B && j != T) ? fx : ex) : 0.f;
      fY[cj][ci] = ey_ok(i, j) ? ((filt && i != L && i != R) ? fy : ey) : 0.f;
    }
  };
  if (filt) laplace(rX, rY, -7, -6, Q1W, Q1H);
#pragma unroll
  for (int q = 0; q < ND; q++) {
    const int k = tid + q * NT;
    if (k < D1H * D1W) {
      const int ci = k % D1W, cj = k / D1W;
      sN[cj][ci] = nd_ok(i0 - 4 + ci, j0 - 4 + cj) ? pn[q] : 0.f;
    }
  }
  if constexpr (LOCAL) {  // coarse E after the coarse step (base_* as the base level)
    float v;
    const float S = A.cS, c1 = A.cc1;
    if (cg <= 1) {
      const int ic = cx0 + cc;
      float hp = base_hz(q[7], S, q[4], q[3], q[1], q[0]);
      if (ic == A.cis - 1) hp += S * cey_src;
      float h = base_hz(q[8], S, q[6], q[5], q[2], q[1]);
      if (ic == A.cis - 1) h += S * cey_src;
      const float kap = base_kap(A.ckn, q[10], q[11]);
      v = base_ex(q[1], kap, S, h, hp, c1, q[9]);
    } else {
      const int I = cg == 3 ? (R >> RS) : (L >> RS);
      float h = base_hz(q[8], S, q[2], q[1], q[6], q[5]);
      if (I == A.cis - 1) h += S * cey_src;
      float hl = base_hz(q[7], S, q[1], q[0], q[4], q[3]);
      if (I - 1 == A.cis - 1) hl += S * cey_src;
      float curl = -S * (h - hl);
      if (I == A.cis) curl += S * chz_src;
      const float kap = base_kap(A.ckn, q[10], q[11]);
      v = base_ey(q[1], kap, curl, c1, q[9]);
    }
    sC[cg < 0 ? 4 : cg][cg < 0 ? 0 : cc] = v;
  } else {  // every thread writes (row 4 is a dummy), so the loads above stay put
    sB1[g1 < 0 ? 4 : g1][g1 < 0 ? 0 : c1_] = ok1 ? cfb(w1a, w1b, b1v0, b1v1, b1v2, b1v3, frac1) : 0.f;
    sB2[g2 < 0 ? 4 : g2][g2 < 0 ? 0 : c2] = ok2 ? cfb(w2a, w2b, b2v0, b2v1, b2v2, b2v3, frac2) : 0.f;
  }
  __syncthreads();
  if constexpr (LOCAL) {  // Eq. (5b) values from the old coarse E and sC
    const int x1 = g1 >= 2 ? cy0 : cx0, x2 = g2 >= 2 ? cy0 : cx0;
    const int r1 = g1 < 0 ? 4 : g1, r2 = g2 < 0 ? 4 : g2;
    const float n1a = ok1 ? sC[r1][k1 - x1] : 0.f, n1b = ok1 ? sC[r1][k1 + 1 - x1] : 0.f;
    const float n2a = ok2 ? sC[r2][k2 - x2] : 0.f, n2b = ok2 ? sC[r2][k2 + 1 - x2] : 0.f;
    sB1[r1][g1 < 0 ? 0 : c1_] = ok1 ? cfb(w1a, w1b, b1v0, b1v1, n1a, n1b, frac1) : 0.f;
    sB2[r2][g2 < 0 ? 0 : c2] = ok2 ? cfb(w2a, w2b, b2v0, b2v1, n2a, n2b, frac2) : 0.f;
  }

  filtered(rX, rY, -7, -5, F1W, F1H);
  __syncthreads();

  // Faraday, H1 over origin -5
#pragma unroll
  for (int q = 0; q < NH0; q++) {
    const int k = tid + q * NT;
    if (k < H1H * H1W) {
      const int ci = k % H1W, cj = k / H1W;
      const int i = i0 - 5 + ci, j = j0 - 5 + cj;
      const float y1 = fY[cj][ci + 1], y0 = fY[cj][ci], x1 = fX[cj + 1][ci], x0 = fX[cj][ci];
      const float dey = y1 - y0;
      const float dex = x1 - x0;
      sH1[cj][ci] = hz_ok(i, j) ? faraday(phz[q], A.S, dey, dex) : 0.f;
    }
  }
  __syncthreads();

  // Ampere + Drude, E1 / J1 over origin -4
#pragma unroll
  for (int q = 0; q < NJ0; q++) {
    const int k = tid + q * NT;
    if (k < N1H * N1W) {
      const int ci = k % N1W, cj = k / N1W;
      const int i = i0 - 4 + ci, j = j0 - 4 + cj;
      // J1 is kept over substep 2's new-E region (origin -1)
      const bool keep = ci >= 3 && cj >= 3 && ci - 3 < N2W && cj - 3 < N2H;
      // every read first (one LDS round trip), then the selects
      const float ex = fX[cj + 1][ci + 1], ey = fY[cj + 1][ci + 1];
      const float n00 = sN[cj][ci], n10 = sN[cj][ci + 1], n01 = sN[cj + 1][ci];
      const float h11 = sH1[cj + 1][ci + 1], h10 = sH1[cj][ci + 1], h01 = sH1[cj + 1][ci];
      const float bx = sB1[j == B ? 0 : 1][ci], by = sB1[i == L ? 2 : 3][cj];
      const bool xok = ex_ok(i, j), yok = ey_ok(i, j);
      const float nex = 0.5f * (n00 + n10);
      const float kx = A.kn * nex;
      const float jox = pjx[q];
      const float dhx = h11 - h10;
      const float ax = ampere(ex, kx, A.S * dhx, A.c1, jox);
      const float exn = xok ? ((j != B && j != T) ? ax : bx) : 0.f;
      if (keep && xok) j1X[cj - 3][ci - 3] = drude(A.a, jox, kx, ex, exn);
      const float ney = 0.5f * (n00 + n01);
      const float ky = A.kn * ney;
      const float joy = pjy[q];
      const float dhy = h11 - h01;
      const float ay = ampere(ey, ky, -A.S * dhy, A.c1, joy);
      const float eyn = yok ? ((i != L && i != R) ? ay : by) : 0.f;
      if (keep && yok) j1Y[cj - 3][ci - 3] = drude(A.a, joy, ky, ey, eyn);
      e1X[cj][ci] = exn;
      e1Y[cj][ci] = eyn;
    }
  }
  __syncthreads();

  // window after substep 1 at the tile's nodes (E1 origin -4)
  float acc1[NA];
#pragma unroll
  for (int q = 0; q < NA; q++) {
    const int r = min(ty + q * RP, TY - 1);  // rows past the tile: discarded
    const int i = i0 + tx, j = j0 + r;
    const int ci = tx + 4, cj = r + 4;
    const float vl = e1X[cj][ci - 1], vr = e1X[cj][ci], vd = e1Y[cj - 1][ci], vu = e1Y[cj][ci];
    float sx = 0.f, sy = 0.f;
    int cx = 0, cy = 0;
    if (i > L) { sx += vl * vl; cx++; }
    if (i < R) { sx += vr * vr; cx++; }
    if (j > B) { sy += vd * vd; cy++; }
    if (j < T) { sy += vu * vu; cy++; }
    acc1[q] = pacc[q] + win_e2(sx, cx, sy, cy);
  }

  // -- substep 2: filter of E1 (raw = E1 at origin -4) -------------------------
  auto laplace2 = [&]() {
    for (int k = tid; k < Q2H * Q2W; k += NT) {
      const int ci = k % Q2W, cj = k / Q2W;
      const int i = i0 - 3 + ci, j = j0 - 3 + cj;
      const int a = ci + 1, b = cj + 1;
      const float xc = e1X[b][a], xl = e1X[b][a - 1], xr = e1X[b][a + 1], xd = e1X[b - 1][a],
                  xu = e1X[b + 1][a];
      const float yc = e1Y[b][a], yl = e1Y[b][a - 1], yr = e1Y[b][a + 1], yd = e1Y[b - 1][a],
                  yu = e1Y[b + 1][a];
      const float lx = lap5(xc, ex_ok(i - 1, j) ? xl : xc, ex_ok(i + 1, j) ? xr : xc,
                            ex_ok(i, j - 1) ? xd : xc, ex_ok(i, j + 1) ? xu : xc);
      const float ly = lap5(yc, ey_ok(i - 1, j) ? yl : yc, ey_ok(i + 1, j) ? yr : yc,
                            ey_ok(i, j - 1) ? yd : yc, ey_ok(i, j + 1) ? yu : yc);
      qX[cj][ci] = ex_ok(i, j) ? lx : 0.f;
      qY[cj][ci] = ey_ok(i, j) ? ly : 0.f;
    }
  };
  if (filt) {
    laplace2();
    __syncthreads();
  }
  for (int k = tid; k < F2H * F2W; k += NT) {
    const int ci = k % F2W, cj = k / F2W;
    const int i = i0 - 2 + ci, j = j0 - 2 + cj;
    const int a = ci + 1, b = cj + 1;  // Laplacian coordinates (origin -3)
    const float ex = e1X[cj + 2][ci + 2], ey = e1Y[cj + 2][ci + 2];
    const float xc = qX[b][a], xl = qX[b][a - 1], xr = qX[b][a + 1], xd = qX[b - 1][a],
                xu = qX[b + 1][a];
    const float yc = qY[b][a], yl = qY[b][a - 1], yr = qY[b][a + 1], yd = qY[b - 1][a],
                yu = qY[b + 1][a];
    const float fx = filter_e(ex, A.gamma,
                              lap5(xc, ex_ok(i - 1, j) ? xl : xc, ex_ok(i + 1, j) ? xr : xc,
                                   ex_ok(i, j - 1) ? xd : xc, ex_ok(i, j + 1) ? xu : xc));
    const float fy = filter_e(ey, A.gamma,
                              lap5(yc, ey_ok(i - 1, j) ? yl : yc, ey_ok(i + 1, j) ? yr : yc,
                                   ey_ok(i, j - 1) ? yd : yc, ey_ok(i, j + 1) ? yu : yc));
    fX[cj][ci] = ex_ok(i, j) ? ((filt && j != B && j != T) ? fx : ex) : 0.f;
    fY[cj][ci] = ey_ok(i, j) ? ((filt && i != L && i != R) ? fy : ey) : 0.f;
  }
  __syncthreads();

  // Faraday, H2 over origin -2 (H1 there at offset 3 in sH1)
  for (int k = tid; k < H2H * H2W; k += NT) {
    const int ci = k % H2W, cj = k / H2W;
    const int i = i0 - 2 + ci, j = j0 - 2 + cj;
    const float y1 = fY[cj][ci + 1], y0 = fY[cj][ci], x1 = fX[cj + 1][ci], x0 = fX[cj][ci];
    const float ho = sH1[cj + 3][ci + 3];
    const float dey = y1 - y0;
    const float dex = x1 - x0;
    const float h = hz_ok(i, j) ? faraday(ho, A.S, dey, dex) : 0.f;
    if (hz_ok(i, j) && ci >= 2 && cj >= 2) sto(tb.hz1, ob(i, j), h);
    sH2[cj][ci] = h;
  }
  __syncthreads();

  // Ampere + Drude, E2 / J2 over origin -1 (n at offset 3, J1 at offset 0)
  for (int k = tid; k < N2H * N2W; k += NT) {
    const int ci = k % N2W, cj = k / N2W;
    const int i = i0 - 1 + ci, j = j0 - 1 + cj;
    const bool own = ci >= 1 && cj >= 1;
    const unsigned o = ob(i, j);
    const float ex = fX[cj + 1][ci + 1], ey = fY[cj + 1][ci + 1];
    const float n00 = sN[cj + 3][ci + 3], n10 = sN[cj + 3][ci + 4], n01 = sN[cj + 4][ci + 3];
    const float h11 = sH2[cj + 1][ci + 1], h10 = sH2[cj][ci + 1], h01 = sH2[cj + 1][ci];
    const float jox = j1X[cj][ci], joy = j1Y[cj][ci];
    const float bx = sB2[j == B ? 0 : 1][ci], by = sB2[i == L ? 2 : 3][cj];
    const bool xok = ex_ok(i, j), yok = ey_ok(i, j);
    const float nex = 0.5f * (n00 + n10);
    const float kx = A.kn * nex;
    const float dhx = h11 - h10;
    const float ax = ampere(ex, kx, A.S * dhx, A.c1, jox);
    const float exn = xok ? ((j != B && j != T) ? ax : bx) : 0.f;
    if (xok && own) {
      const float jn = drude(A.a, jox, kx, ex, exn);
      sto(tb.ex1, o, exn);
      sto(tb.jx1, o, jn);
      j2X[cj - 1][ci - 1] = jn;
    }
    const float ney = 0.5f * (n00 + n01);
    const float ky = A.kn * ney;
    const float dhy = h11 - h01;
    const float ay = ampere(ey, ky, -A.S * dhy, A.c1, joy);
    const float eyn = yok ? ((i != L && i != R) ? ay : by) : 0.f;
    if (yok && own) {
      const float jn = drude(A.a, joy, ky, ey, eyn);
      sto(tb.ey1, o, eyn);
      sto(tb.jy1, o, jn);
      j2Y[cj - 1][ci - 1] = jn;
    }
    e2X[cj][ci] = exn;
    e2Y[cj][ci] = eyn;
  }
  __syncthreads();

  // window after substep 2
#pragma unroll
  for (int q = 0; q < NA; q++) {
    const int r = ty + q * RP;
    const int i = i0 + tx, j = j0 + r;
    if (r >= TY || !nd_ok(i, j)) continue;
    const int ci = tx + 1, cj = r + 1;
    const float vl = e2X[cj][ci - 1], vr = e2X[cj][ci], vd = e2Y[cj - 1][ci], vu = e2Y[cj][ci];
    float sx = 0.f, sy = 0.f;
    int cx = 0, cy = 0;
    if (i > L) { sx += vl * vl; cx++; }
    if (i < R) { sx += vr * vr; cx++; }
    if (j > B) { sy += vd * vd; cy++; }
    if (j < T) { sy += vu * vu; cy++; }
    sto(tb.acc, ob(i, j), acc1[q] + win_e2(sx, cx, sy, cy));
  }

  // fine -> coarse transfer (H1 at origin -5, H2 at origin -2)
  if constexpr (R4) {
    // 4 x 4 cells at the half levels after substeps 2 (the input Hz) and 3
    // (H1); 4 edges, J~ summed
    if (A.restrict_on) {
      for (int r = ty; r < TY; r += RP) {
        const int i = i0 + tx, j = j0 + r;
        if (((i - L) | (j - B)) & 3) continue;
        const int a = i >> 2, b = j >> 2;
        const size_t co = (size_t)b * A.cpitch + a;
        const int ci = tx + 1, cj = r + 1;
        if (hz_ok(i, j)) {
          float s = 0.f;
          for (int da = 0; da < 4; da++)
            for (int db = 0; db < 4; db++) {
              const float lo = A.hz0[(size_t)(j + db) * pitch + i + da];
              s += 0.5f * (lo + sH1[r + 5 + db][tx + 5 + da]);
            }
          A.chz[co] = 0.0625f * s;
        }
        if (ex_ok(i, j) && j > B && j < T) {
          float se = 0.f, sj = 0.f;
          for (int da = 0; da < 4; da++) { se += e2X[cj][ci + da]; sj += j2X[r][tx + da]; }
          A.cex[co] = 0.25f * se;
          A.cjx[co] = sj;
        }
        if (ey_ok(i, j) && i > L && i < R) {
          float se = 0.f, sj = 0.f;
          for (int db = 0; db < 4; db++) { se += e2Y[cj + db][ci]; sj += j2Y[r + db][tx]; }
          A.cey[co] = 0.25f * se;
          A.cjy[co] = sj;
        }
      }
    }
  } else {
    for (int r = ty; r < TY; r += RP) {
      const int i = i0 + tx, j = j0 + r;
      if (((i - L) | (j - B)) & 1) continue;
      const int a = i >> 1, b = j >> 1;
      const size_t co = (size_t)b * A.cpitch + a;
      const int ci = tx + 1, cj = r + 1;
      if (hz_ok(i, j)) {
        float s = 0.f;
        for (int da = 0; da < 2; da++)
          for (int db = 0; db < 2; db++) {
            const float hold = sH1[r + 5 + db][tx + 5 + da];
            s += 0.5f * (hold + sH2[r + 2 + db][tx + 2 + da]);
          }
        A.chz[co] = 0.25f * s;
      }
      if (ex_ok(i, j) && j > B && j < T) {
        A.cex[co] = 0.5f * (e2X[cj][ci] + e2X[cj][ci + 1]);
        A.cjx[co] = j2X[r][tx] + j2X[r][tx + 1];  // J~ scales with dt
      }
      if (ey_ok(i, j) && i > L && i < R) {
        A.cey[co] = 0.5f * (e2Y[cj][ci] + e2Y[cj + 1][ci]);
        A.cjy[co] = j2Y[r][tx] + j2Y[r + 1][tx];
      }
    }
  }

  // replay for the adjoint: E entering (raw E0 at origin -7), after
  // substep 1 (origin -4), after substep 2 (origin -1), n (origin -4)
  if constexpr (ST) {
    for (int r = ty; r < TY; r += RP) {
      const int i = i0 + tx, j = j0 + r;
      if (!nd_ok(i, j)) continue;
      const size_t o = (size_t)j * pitch + i;
      A.stn[o] = sN[r + 4][tx + 4];
      if (ex_ok(i, j)) {
        A.st0x[o] = rX[r + 7][tx + 7];
        A.st1x[o] = e1X[r + 4][tx + 4];
        if (A.st2x) A.st2x[o] = e2X[r + 1][tx + 1];
      }
      if (ey_ok(i, j)) {
        A.st0y[o] = rY[r + 7][tx + 7];
        A.st1y[o] = e1Y[r + 4][tx + 4];
        if (A.st2y) A.st2y[o] = e2Y[r + 1][tx + 1];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Both patch substeps of the combined step (rectangle, patch tiles computing
// the coarse boundary E themselves), laid out for short phases.  R4: a pair
// of the four r = 4 substeps (the first inside the base step's launch, the
// second, with the r = 4 fine -> coarse transfer, in k_fine2_fast).
// Every array of the tile lives in one LDS frame, the raw-E region of the
// first substep (origin (-7, -7) from the tile corner, FW x FH), and each
// thread owns fixed frame positions for the whole launch: their coordinates,
// validity and clamped positions are formed once, and every phase reads its
// neighbours at constant offsets.  Entities outside the patch hold the value
// of the nearest entity inside it: raw E and J come from clamped addresses,
// and the Laplacians and the first substep's new E are formed at the clamped
// position.  That is the filter's zero-gradient rule at the patch edge, so no
// phase tests its neighbours.  Every entity is computed with the operations
// and operands of fine2_tile (the helpers above), so the results are
// identical to it and to two one-substep launches.
// ---------------------------------------------------------------------------
template <int TY, int NT, int TW, bool R4 = false>
__device__ __forceinline__ void fine2_fast(const EMArgs& A, int bx, int by, float cey_src,
                                           float chz_src) {
  constexpr int FW = TW + 13, FH = TY + 13, FN = FW * FH;
  constexpr int NP = (FN + NT - 1) / NT;  // frame positions per thread
  __shared__ float rX[FN], rY[FN];    // raw E0 (clamped)
  __shared__ float fX[FN], fY[FN];    // filtered E0, then filtered E1
  __shared__ float sH0[FN], sH1[FN], sH2[FN];  // Hz entering, after substeps 1 and 2
  __shared__ float e1X[FN], e1Y[FN];  // E1 (at clamped positions)
  __shared__ float e2X[FN], e2Y[FN];  // E2
  __shared__ float j2X[FN], j2Y[FN];  // J2 of the tile's own edges
  __shared__ float sN[FN];
  constexpr int CW = TW / 2 + 6, CH = TY / 2 + 6;
  __shared__ float sC[5][CW > CH ? CW : CH];  // coarse E on the boundary lines after the step
  __shared__ float sO[5][CW > CH ? CW : CH];  // and before it

  const int i0 = A.L + bx * TW;
  const int j0 = A.B + by * TY;
  const int tid = threadIdx.x;
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const bool filt = A.gamma > 0.f;
  const float frac1 = A.frac, frac2 = R4 ? A.frac + 0.25f : 1.f;
  const int ib = max(i0 - 8, L), jb = max(j0 - 8, B);
  const TileBase tb(A, ib, jb);
  auto cl = [=](int v, int lo, int hi) { return min(max(v, lo), hi); };
  const int fi0 = i0 - 7, fj0 = j0 - 7;  // physical position of frame entry 0

  // -- per position: frame offset, flags, clamped offsets; issue every load
  int po[NP], ci_[NP], cj_[NP], ocx[NP], ocy[NP], cxi[NP], cxj[NP], cyi[NP], cyj[NP];
  bool inf[NP], hzok[NP], exok[NP], eyok[NP], ndok[NP];
  float pex[NP], pey[NP], phz[NP], pjx[NP], pjy[NP], pn[NP], pacc[NP];
#pragma unroll
  for (int q = 0; q < NP; q++) {
    const int p = tid + q * NT;
    inf[q] = p < FN;
    const int pp = inf[q] ? p : FN - 1;
    po[q] = pp;
    const int ci = pp % FW, cj = pp / FW;
    ci_[q] = ci; cj_[q] = cj;
    const int i = fi0 + ci, j = fj0 + cj;
    hzok[q] = i >= L && i < R && j >= B && j < T;
    exok[q] = i >= L && i < R && j >= B && j <= T;
    eyok[q] = i >= L && i <= R && j >= B && j < T;
    ndok[q] = i >= L && i <= R && j >= B && j <= T;
    const int ixc = cl(i, L, R - 1), jxc = cl(j, B, T);
    const int iyc = cl(i, L, R), jyc = cl(j, B, T - 1);
    ocx[q] = (jxc - fj0) * FW + (ixc - fi0);
    ocy[q] = (jyc - fj0) * FW + (iyc - fi0);
    cxi[q] = ixc; cxj[q] = jxc; cyi[q] = iyc; cyj[q] = jyc;
    const unsigned ox = tb.off(ixc, jxc), oy = tb.off(iyc, jyc);
    const unsigned oh = tb.off(cl(i, L, R - 1), cl(j, B, T - 1));
    const unsigned on = tb.off(cl(i, L, R), cl(j, B, T));
    pex[q] = ldo(tb.ex0, ox);
    pey[q] = ldo(tb.ey0, oy);
    phz[q] = ldo(tb.hz0, oh);
    pjx[q] = ldo(tb.jx0, ox);
    pjy[q] = ldo(tb.jy0, oy);
    pn[q] = ldo(tb.n, on);
    pacc[q] = 0.f;
    if (ci >= 7 && ci < 7 + TW && cj >= 7 && cj < 7 + TY) pacc[q] = ldo(tb.acc, on);
  }
  // coarse state around the patch boundary lines, for the coarse E after the
  // step there (as in fine2_tile)
  constexpr int RS = R4 ? 2 : 1;  // fine -> coarse index shift
  const int cx0 = ((i0 - 4) >> RS) - 1, cy0 = ((j0 - 4) >> RS) - 1;
  int cg = -1, cc = 0;
  float qc[12];
  if (tid < CW) { cg = 0; cc = tid; }
  else if (tid < 2 * CW) { cg = 1; cc = tid - CW; }
  else if (tid < 2 * CW + CH) { cg = 2; cc = tid - 2 * CW; }
  else if (tid < 2 * CW + 2 * CH) { cg = 3; cc = tid - 2 * CW - CH; }
  {
    const unsigned cp4 = (unsigned)A.cpitch * 4u;
    const int NXc = A.cnx, NYc = A.cny;
    auto cidx = [=](int a, int b) {  // clamped coarse byte offset
      const int aa = a < 0 ? 0 : (a > NXc ? NXc : a), bb = b < 0 ? 0 : (b > NYc ? NYc : b);
      return __umul24((unsigned)bb, cp4) + ((unsigned)aa << 2);
    };
    if (cg <= 1) {  // x-edge (ic, J) of a boundary row (threads without a role: cg = -1)
      const int ic = cx0 + cc, J = cg == 1 ? (T >> RS) : (B >> RS);
      qc[0] = ldo(A.cex0, cidx(ic, J - 1)); qc[1] = ldo(A.cex0, cidx(ic, J));
      qc[2] = ldo(A.cex0, cidx(ic, J + 1));
      qc[3] = ldo(A.cey0, cidx(ic, J - 1)); qc[4] = ldo(A.cey0, cidx(ic + 1, J - 1));
      qc[5] = ldo(A.cey0, cidx(ic, J)); qc[6] = ldo(A.cey0, cidx(ic + 1, J));
      qc[7] = ldo(A.chz0, cidx(ic, J - 1)); qc[8] = ldo(A.chz0, cidx(ic, J));
      qc[9] = ldo(A.cjx0, cidx(ic, J)); qc[10] = ldo(A.cn0, cidx(ic, J));
      qc[11] = ldo(A.cn0, cidx(ic + 1, J));
    } else {        // y-edge (I, jc) of a boundary column
      const int jc = cy0 + cc, I = cg == 3 ? (R >> RS) : (L >> RS);
      qc[0] = ldo(A.cey0, cidx(I - 1, jc)); qc[1] = ldo(A.cey0, cidx(I, jc));
      qc[2] = ldo(A.cey0, cidx(I + 1, jc));
      qc[3] = ldo(A.cex0, cidx(I - 1, jc)); qc[4] = ldo(A.cex0, cidx(I - 1, jc + 1));
      qc[5] = ldo(A.cex0, cidx(I, jc)); qc[6] = ldo(A.cex0, cidx(I, jc + 1));
      qc[7] = ldo(A.chz0, cidx(I - 1, jc)); qc[8] = ldo(A.chz0, cidx(I, jc));
      qc[9] = ldo(A.cjy0, cidx(I, jc)); qc[10] = ldo(A.cn0, cidx(I, jc));
      qc[11] = ldo(A.cn0, cidx(I, jc + 1));
    }
  }
  // region tests in frame coordinates (origin o, width TW + w, height TY + h)
  auto in_reg = [](int ci, int cj, int o, int w, int h) {
    const int a = ci - 7 - o, b = cj - 7 - o;
    return a >= 0 && a < TW + w && b >= 0 && b < TY + h;
  };
  auto own = [](int ci, int cj) { return ci >= 7 && ci < 7 + TW && cj >= 7 && cj < 7 + TY; };

  // -- raw E0 (clamped values: entities outside the patch hold their nearest
  // entity's value)
#pragma unroll
  for (int q = 0; q < NP; q++)
    if (inf[q]) { rX[po[q]] = pex[q]; rY[po[q]] = pey[q]; }
  __syncthreads();

  // L(L(E)) of the filter at frame offset p of a padded field x: the
  // Laplacian at p and at its four neighbours, a neighbour outside the patch
  // replaced by p itself (zero gradient at the patch edge); the same
  // Laplacians, in the same order, as forming them in a phase of their own
  auto lap2 = [](const float* x, int p, bool lv, bool rv, bool dv, bool uv) {
    const float c = x[p], l1 = x[p - 1], r1 = x[p + 1], d1 = x[p - FW], u1 = x[p + FW];
    const float l2 = x[p - 2], r2 = x[p + 2], d2 = x[p - 2 * FW], u2 = x[p + 2 * FW];
    const float ld = x[p - 1 - FW], lu = x[p - 1 + FW], rd = x[p + 1 - FW], ru = x[p + 1 + FW];
    const float Lc = lap5(c, l1, r1, d1, u1);
    const float Ll = lap5(l1, l2, c, ld, lu);
    const float Lr = lap5(r1, c, r2, rd, ru);
    const float Ld = lap5(d1, ld, rd, d2, c);
    const float Lu = lap5(u1, lu, ru, c, u2);
    return lap5(Lc, lv ? Ll : Lc, rv ? Lr : Lc, dv ? Ld : Lc, uv ? Lu : Lc);
  };
  // Eq. (5b) value of the boundary edge at position e along line g (0/1:
  // x-edges of rows B/T, 2/3: y-edges of columns L/R) from the coarse E on
  // the line before (sO) and after (sC) the coarse step; offsets 1/4, 3/4
  // (r = 4: 1/8 ... 7/8, lower coarse edge and weights as in bnd_src)
  constexpr int SW = CW > CH ? CW : CH;
  auto cfb_at = [=](int g, int e, float fr) {
    int k;
    float w0, w1;
    if constexpr (R4) {
      const int m = e & 3;
      k = (e >> 2) - (m < 2 ? 1 : 0);
      w0 = m == 0 ? 0.375f : m == 1 ? 0.125f : m == 2 ? 0.875f : 0.625f;
      w1 = 1.f - w0;
    } else {
      const bool ev = (e & 1) == 0;
      k = ev ? (e >> 1) - 1 : (e >> 1);
      w0 = ev ? 0.25f : 0.75f;
      w1 = ev ? 0.75f : 0.25f;
    }
    const int x = min(max(k - (g >= 2 ? cy0 : cx0), 0), SW - 2);
    return cfb(w0, w1, sO[g][x], sO[g][x + 1], sC[g][x], sC[g][x + 1], fr);
  };
  const float S = A.S;

  // -- phase A: n, old Hz, coarse E after the step on the boundary lines;
  // filtered E0 over origin -5
#pragma unroll
  for (int q = 0; q < NP; q++)
    if (inf[q]) { sN[po[q]] = ndok[q] ? pn[q] : 0.f; sH0[po[q]] = phz[q]; }
  {
    float v;
    const float cS = A.cS, c1 = A.cc1;
    if (cg <= 1) {
      const int ic = cx0 + cc;
      float hp = base_hz(qc[7], cS, qc[4], qc[3], qc[1], qc[0]);
      if (ic == A.cis - 1) hp += cS * cey_src;
      float h = base_hz(qc[8], cS, qc[6], qc[5], qc[2], qc[1]);
      if (ic == A.cis - 1) h += cS * cey_src;
      const float kap = base_kap(A.ckn, qc[10], qc[11]);
      v = base_ex(qc[1], kap, cS, h, hp, c1, qc[9]);
    } else {
      const int I = cg == 3 ? (R >> RS) : (L >> RS);
      float h = base_hz(qc[8], cS, qc[2], qc[1], qc[6], qc[5]);
      if (I == A.cis - 1) h += cS * cey_src;
      float hl = base_hz(qc[7], cS, qc[1], qc[0], qc[4], qc[3]);
      if (I - 1 == A.cis - 1) hl += cS * cey_src;
      float curl = -cS * (h - hl);
      if (I == A.cis) curl += cS * chz_src;
      const float kap = base_kap(A.ckn, qc[10], qc[11]);
      v = base_ey(qc[1], kap, curl, c1, qc[9]);
    }
    sC[cg < 0 ? 4 : cg][cg < 0 ? 0 : cc] = v;
    sO[cg < 0 ? 4 : cg][cg < 0 ? 0 : cc] = qc[1];  // the line's own coarse E entering
  }
#pragma unroll
  for (int q = 0; q < NP; q++) {
    if (!(inf[q] && in_reg(ci_[q], cj_[q], -5, 9, 9))) continue;
    const int p = po[q], j = fj0 + cj_[q], i = fi0 + ci_[q];
    const float ex = rX[p], ey = rY[p];
    float fx = ex, fy = ey;
    if (filt) {
      if (j != B && j != T) fx = filter_e(ex, A.gamma, lap2(rX, p, i > L, i < R - 1, j > B, j < T));
      if (i != L && i != R) fy = filter_e(ey, A.gamma, lap2(rY, p, i > L, i < R, j > B, j < T - 1));
    }
    fX[p] = exok[q] ? fx : 0.f;
    fY[p] = eyok[q] ? fy : 0.f;
  }
  __syncthreads();

  // -- phase B: substep 1, Faraday and Ampere + Drude together.  E1 over
  // origin -4 at the clamped positions, from the H1 of the cells beside the
  // edge (formed here); the cell's own H1 kept for substep 2 and the
  // transfer; J1 of the entities substep 2 updates in registers
  auto far1 = [=](int c, bool ok) {
    const float y1 = fY[c + 1], y0 = fY[c], x1 = fX[c + FW], x0 = fX[c], ho = sH0[c];
    const float dey = y1 - y0;
    const float dex = x1 - x0;
    return ok ? faraday(ho, S, dey, dex) : 0.f;
  };
  float j1x[NP], j1y[NP];
#pragma unroll
  for (int q = 0; q < NP; q++) {
    j1x[q] = 0.f; j1y[q] = 0.f;
    if (!(inf[q] && in_reg(ci_[q], cj_[q], -4, 7, 7))) continue;
    const int p = po[q];
    const int ox = ocx[q], oy = ocy[q];
    const int ixc = cxi[q], jxc = cxj[q], iyc = cyi[q], jyc = cyj[q];
    const float hx1 = far1(ox, jxc < T), hx0 = far1(ox - FW, jxc > B);
    const float hy1 = far1(oy, iyc < R), hy0 = far1(oy - 1, iyc > L);
    const float ex = fX[ox], ey = fY[oy];
    const float nx0 = sN[ox], nx1 = sN[ox + 1], ny0 = sN[oy], ny1 = sN[oy + FW];
    const float bx = cfb_at(jxc == T ? 1 : 0, ixc, frac1);
    const float by = cfb_at(iyc == R ? 3 : 2, jyc, frac1);
    const float nex = 0.5f * (nx0 + nx1);
    const float kx = A.kn * nex;
    const float dhx = hx1 - hx0;
    const float ax = ampere(ex, kx, S * dhx, A.c1, pjx[q]);
    const float exn = (jxc != B && jxc != T) ? ax : bx;
    const float ney = 0.5f * (ny0 + ny1);
    const float ky = A.kn * ney;
    const float dhy = hy1 - hy0;
    const float ay = ampere(ey, ky, -S * dhy, A.c1, pjy[q]);
    const float eyn = (iyc != L && iyc != R) ? ay : by;
    e1X[p] = exn;
    e1Y[p] = eyn;
    j1x[q] = drude(A.a, pjx[q], kx, ex, exn);
    j1y[q] = drude(A.a, pjy[q], ky, ey, eyn);
    sH1[p] = hzok[q] ? hx1 : 0.f;  // a valid cell is its own x-edge's (ox == p)
  }
  __syncthreads();

  // -- phase C: window after substep 1 at the tile's own nodes (registers);
  // filtered E1 over origin -2
  float acc1[NP];
#pragma unroll
  for (int q = 0; q < NP; q++) {
    acc1[q] = 0.f;
    if (!(inf[q] && own(ci_[q], cj_[q]))) continue;
    const int p = po[q], i = fi0 + ci_[q], j = fj0 + cj_[q];
    const float vl = e1X[p - 1], vr = e1X[p], vd = e1Y[p - FW], vu = e1Y[p];
    float sx = 0.f, sy = 0.f;
    int cx = 0, cy = 0;
    if (i > L) { sx += vl * vl; cx++; }
    if (i < R) { sx += vr * vr; cx++; }
    if (j > B) { sy += vd * vd; cy++; }
    if (j < T) { sy += vu * vu; cy++; }
    acc1[q] = pacc[q] + win_e2(sx, cx, sy, cy);
  }
#pragma unroll
  for (int q = 0; q < NP; q++) {
    if (!(inf[q] && in_reg(ci_[q], cj_[q], -2, 3, 3))) continue;
    const int p = po[q], j = fj0 + cj_[q], i = fi0 + ci_[q];
    const float ex = e1X[p], ey = e1Y[p];
    float fx = ex, fy = ey;
    if (filt) {
      if (j != B && j != T) fx = filter_e(ex, A.gamma, lap2(e1X, p, i > L, i < R - 1, j > B, j < T));
      if (i != L && i != R) fy = filter_e(ey, A.gamma, lap2(e1Y, p, i > L, i < R, j > B, j < T - 1));
    }
    fX[p] = exok[q] ? fx : 0.f;
    fY[p] = eyok[q] ? fy : 0.f;
  }
  __syncthreads();

  // -- phase D: substep 2, Faraday and Ampere + Drude together over origin
  // -1; the tile's own entities stored
  auto far2 = [=](int c, bool ok) {
    const float y1 = fY[c + 1], y0 = fY[c], x1 = fX[c + FW], x0 = fX[c], ho = sH1[c];
    const float dey = y1 - y0;
    const float dex = x1 - x0;
    return ok ? faraday(ho, S, dey, dex) : 0.f;
  };
#pragma unroll
  for (int q = 0; q < NP; q++) {
    if (!(inf[q] && in_reg(ci_[q], cj_[q], -1, 1, 1))) continue;
    const int p = po[q], i = fi0 + ci_[q], j = fj0 + cj_[q];
    const bool ow = own(ci_[q], cj_[q]);
    const unsigned o = tb.off(i, j);
    const bool cin = i >= L && i < R;  // column of cells inside the patch
    const float h11 = far2(p, hzok[q]);
    const float h10 = far2(p - FW, cin && j - 1 >= B && j - 1 < T);
    const float h01 = far2(p - 1, i - 1 >= L && i - 1 < R && j >= B && j < T);
    if (hzok[q] && ow) sto(tb.hz1, o, h11);
    sH2[p] = h11;
    const float ex = fX[p], ey = fY[p];
    const float n00 = sN[p], n10 = sN[p + 1], n01 = sN[p + FW];
    const float bx = cfb_at(j == T ? 1 : 0, i, frac2), by = cfb_at(i == R ? 3 : 2, j, frac2);
    const float nex = 0.5f * (n00 + n10);
    const float kx = A.kn * nex;
    const float dhx = h11 - h10;
    const float ax = ampere(ex, kx, S * dhx, A.c1, j1x[q]);
    const float exn = exok[q] ? ((j != B && j != T) ? ax : bx) : 0.f;
    if (exok[q] && ow) {
      const float jn = drude(A.a, j1x[q], kx, ex, exn);
      sto(tb.ex1, o, exn);
      sto(tb.jx1, o, jn);
      j2X[p] = jn;
    }
    const float ney = 0.5f * (n00 + n01);
    const float ky = A.kn * ney;
    const float dhy = h11 - h01;
    const float ay = ampere(ey, ky, -S * dhy, A.c1, j1y[q]);
    const float eyn = eyok[q] ? ((i != L && i != R) ? ay : by) : 0.f;
    if (eyok[q] && ow) {
      const float jn = drude(A.a, j1y[q], ky, ey, eyn);
      sto(tb.ey1, o, eyn);
      sto(tb.jy1, o, jn);
      j2Y[p] = jn;
    }
    e2X[p] = exn;
    e2Y[p] = eyn;
  }
  __syncthreads();

  // -- window after substep 2 and the fine -> coarse transfer, own nodes
#pragma unroll
  for (int q = 0; q < NP; q++) {
    if (!(inf[q] && own(ci_[q], cj_[q]))) continue;
    const int p = po[q], i = fi0 + ci_[q], j = fj0 + cj_[q];
    if (ndok[q]) {
      const float vl = e2X[p - 1], vr = e2X[p], vd = e2Y[p - FW], vu = e2Y[p];
      float sx = 0.f, sy = 0.f;
      int cx = 0, cy = 0;
      if (i > L) { sx += vl * vl; cx++; }
      if (i < R) { sx += vr * vr; cx++; }
      if (j > B) { sy += vd * vd; cy++; }
      if (j < T) { sy += vu * vu; cy++; }
      sto(tb.acc, tb.off(i, j), acc1[q] + win_e2(sx, cx, sy, cy));
    }
    if constexpr (R4) {
      // r = 4, after the second pair: 4 x 4 cells at the half levels after
      // substeps 2 (the Hz entering) and 3; 4 edges, J~ summed
      if (!A.restrict_on || (((i - L) | (j - B)) & 3)) continue;
      const int a = i >> 2, b = j >> 2;
      const size_t co = (size_t)b * A.cpitch + a;
      if (hzok[q]) {
        float s = 0.f;
        for (int da = 0; da < 4; da++)
          for (int db = 0; db < 4; db++)
            s += 0.5f * (sH0[p + db * FW + da] + sH1[p + db * FW + da]);
        A.chz[co] = 0.0625f * s;
      }
      if (exok[q] && j > B && j < T) {
        float se = 0.f, sj = 0.f;
        for (int da = 0; da < 4; da++) { se += e2X[p + da]; sj += j2X[p + da]; }
        A.cex[co] = 0.25f * se;
        A.cjx[co] = sj;
      }
      if (eyok[q] && i > L && i < R) {
        float se = 0.f, sj = 0.f;
        for (int db = 0; db < 4; db++) { se += e2Y[p + db * FW]; sj += j2Y[p + db * FW]; }
        A.cey[co] = 0.25f * se;
        A.cjy[co] = sj;
      }
      continue;
    }
    if (((i - L) | (j - B)) & 1) continue;
    const int a = i >> 1, b = j >> 1;
    const size_t co = (size_t)b * A.cpitch + a;
    if (hzok[q]) {
      float s = 0.f;
      for (int da = 0; da < 2; da++)
        for (int db = 0; db < 2; db++) {
          const float hold = sH1[p + db * FW + da];
          s += 0.5f * (hold + sH2[p + db * FW + da]);
        }
      A.chz[co] = 0.25f * s;
    }
    if (exok[q] && j > B && j < T) {
      A.cex[co] = 0.5f * (e2X[p] + e2X[p + 1]);
      A.cjx[co] = j2X[p] + j2X[p + 1];  // J~ scales with dt
    }
    if (eyok[q] && i > L && i < R) {
      A.cey[co] = 0.5f * (e2Y[p] + e2Y[p + FW]);
      A.cjy[co] = j2Y[p] + j2Y[p + FW];
    }
  }
}

template <int TY, int NT, bool ST = false, bool R4 = false, int TW = kTX>
__global__ __launch_bounds__(NT) void k_fine2(EMArgs A) {
  fine2_tile<TY, NT, false, ST, R4, TW>(A, blockIdx.x, blockIdx.y, 0.f, 0.f);
}

// Two patch substeps after the base step's own launch, in the frame tile of
// the combined step: r = 2, both substeps and the fine -> coarse transfer;
// R4, the second pair of r = 4 substeps (3, 4) and the transfer.  The tiles
// form the coarse E after the coarse step on their boundary lines from the
// coarse state entering it (its buffers are still intact), as in the
// combined launch.
template <int TW, bool R4>
__global__ __launch_bounds__(step_threads(false, 4)) void k_fine2_fast(EMArgs A) {
  fine2_fast<4, step_threads(false, 4), TW, R4>(A, blockIdx.x, blockIdx.y, A.cey_src, A.chz_src);
}


// batched form: one launch over the tiles of many independent instances;
// blk[b] = (instance, tile index within it)
template <int TY>
__global__ __launch_bounds__(kFineThreads) void k_fine_batch(const EMArgs* __restrict__ args,
                                                             const int2* __restrict__ blk) {
  const int2 bi = blk[blockIdx.x];
  const EMArgs& A = args[bi.x];
  __shared__ FineLds<TY, false> S;
  const int bx = bi.y % A.nbx, by = bi.y / A.nbx;
  if (fine_interior(A, A.L + bx * kTX, A.B + by * TY, TY))
    fine_tile<TY, kFineThreads, false, true>(A, S, bx, by);
  else
    fine_tile<TY, kFineThreads>(A, S, bx, by);
}

// batched two-substep patch launch (both substeps of r = 2, or a pair of the
// four of r = 4), over the same (instance, 64 x TY tile) table
template <int TY, bool R4>
__global__ __launch_bounds__(kFineThreads) void k_fine2_batch(const EMArgs* __restrict__ args,
                                                              const int2* __restrict__ blk) {
  const int2 bi = blk[blockIdx.x];
  const EMArgs& A = args[bi.x];
  fine2_tile<TY, kFineThreads, false, false, R4, kTX>(A, bi.y % A.nbx, bi.y / A.nbx, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// Window block close and continuity step (Eq. (4)), one thread per node of
// the region [L..R] x [B..T].  ring[slot] <- acc / steps_per_period,
// acc <- 0; with `update`, E_rms^2 = sum of the 8 ring slots,
// nu = nu_m A [(E_eff^2/(100p)^2)^(beta/2) - (E_cr/p)^beta] (or the
// Townsend form gamma v_d - nu_att),
// n+ = n + dt_n [dx^-2 sum_faces (D_i+D_nb)/2 (n_nb - n) + (nu - r_ei n) n]  (>= 0).
// Fine level: interior nodes are updated; boundary nodes take the new coarse
// density (copy / mean along the boundary line); the coarse nodes strictly
// inside the patch take the new fine density (injection).
// ---------------------------------------------------------------------------
__device__ inline float d_eff(const ContArgs &A, float n) {
  if (A.d_const_mode) return A.d_const;
  const float al = n * A.inv_namb;
  return (al * A.Da + A.De) / (1.f + al);
}

// the new density of one updated node from its old value, the neighbours
// that exist (zero-flux faces elsewhere) and E_rms^2
__device__ __forceinline__ float cont_update(const ContArgs& A, size_t o, float e2, bool l,
                                             bool r, bool d, bool u) {
  const int pitch = A.pitch;
  const float ni = A.n0[o];
  const float di = d_eff(A, ni);
  float flux = 0.f;
  if (l) { const float v = A.n0[o - 1]; flux += 0.5f * (di + d_eff(A, v)) * (v - ni); }
  if (r) { const float v = A.n0[o + 1]; flux += 0.5f * (di + d_eff(A, v)) * (v - ni); }
  if (d) { const float v = A.n0[o - pitch]; flux += 0.5f * (di + d_eff(A, v)) * (v - ni); }
  if (u) { const float v = A.n0[o + pitch]; flux += 0.5f * (di + d_eff(A, v)) * (v - ni); }
  float nn;
  if (!A.town && A.rei == 0.f) {
    const float nu = A.nuA * (powf(e2 * A.eeff_p2, A.half_beta) - A.att);
    nn = ni + A.dtn * (flux * A.inv_dx2 + nu * ni);
  } else {  // Townsend ionisation and / or recombination
    float nu;
    if (A.town) {
      const float y = sqrtf(e2 * A.eeff_p2);  // E_eff / (100 p), V/(cm Torr)
      nu = (y > 0.f ? A.tK * y * expf(-A.tB / y) : 0.f) - A.tatt;
    } else {
      nu = A.nuA * (powf(e2 * A.eeff_p2, A.half_beta) - A.att);
    }
    nn = ni + A.dtn * (flux * A.inv_dx2 + (nu - A.rei * ni) * ni);
  }
  return nn > 0.f ? nn : 0.f;
}

// MERGED (both levels in one launch, k_cont2): the coarse level leaves the
// nodes on the patch boundary lines to the boundary block and does not
// write the density of nodes strictly inside the patch (the injection
// does); the patch level leaves its boundary nodes to the boundary block.
template <bool FINE, bool MERGED = false, int NT = kThreads>
__device__ __forceinline__ void cont_body(const ContArgs& A, int bx, int by, int slot,
                                          int update) {
  const int i = A.L + bx * kTX + (threadIdx.x % kTX);
  const int j = A.B + by * (NT / kTX) + (threadIdx.x / kTX);
  if (i > A.R || j > A.T) return;
  bool inner = false;  // MERGED coarse level: strictly inside the patch
  if constexpr (MERGED) {
    if constexpr (FINE) {
      if (i == A.L || i == A.R || j == A.B || j == A.T) return;
    } else {
      const bool inx = i >= A.pL && i <= A.pR, iny = j >= A.pB && j <= A.pT;
      if ((inx && (j == A.pB || j == A.pT)) || (iny && (i == A.pL || i == A.pR))) return;
      inner = i > A.pL && i < A.pR && j > A.pB && j < A.pT;
    }
  }
  const int pitch = A.pitch;
  const size_t o = (size_t)j * pitch + i;
  const float sv = A.acc[o] * A.inv_spp;
  A.ring[(size_t)slot * A.plane + o] = sv;
  A.acc[o] = 0.f;
  if (!update) {
    if (!isfinite(sv)) A.err[threadIdx.x & 63] = 1;
    return;
  }
  float e2 = 0.f;
  for (int s = 0; s < kRing; s++)
    e2 += (s == slot) ? sv : A.ring[(size_t)s * A.plane + o];
  float nn;
  if (FINE && A.rf == 4 && (i == A.L || i == A.R || j == A.B || j == A.T)) {
    // linear along the boundary line between the two coarse nodes
    const int a = i >> 2, b = j >> 2, cp = A.cpitch;
    const float ti = (i & 3) * 0.25f, tj = (j & 3) * 0.25f;
    const float c00 = A.cn1[(size_t)b * cp + a];
    if ((i & 3) != 0) nn = (1.f - ti) * c00 + ti * A.cn1[(size_t)b * cp + a + 1];
    else if ((j & 3) != 0) nn = (1.f - tj) * c00 + tj * A.cn1[(size_t)(b + 1) * cp + a];
    else nn = c00;
  } else if (FINE && (i == A.L || i == A.R || j == A.B || j == A.T)) {
    const int a = i >> 1, b = j >> 1, cp = A.cpitch;
    if (((i | j) & 1) == 0) nn = A.cn1[(size_t)b * cp + a];
    else if (i & 1) nn = 0.5f * (A.cn1[(size_t)b * cp + a] + A.cn1[(size_t)b * cp + a + 1]);
    else nn = 0.5f * (A.cn1[(size_t)b * cp + a] + A.cn1[(size_t)(b + 1) * cp + a]);
  } else {
    nn = cont_update(A, o, e2, i > A.L, i < A.R, j > A.B, j < A.T);
    const int rm = A.rf == 4 ? 3 : 1, rs = A.rf == 4 ? 2 : 1;
    if (FINE && (((i - A.L) | (j - A.B)) & rm) == 0) {
      const int a = i >> rs, b = j >> rs;  // strictly inside: coincident node
      A.cn1[(size_t)b * A.cpitch + a] = nn;
    }
  }
  if (inner) return;  // the injection writes it
  A.n1[o] = nn;
  if (!isfinite(nn) || !isfinite(e2)) A.err[threadIdx.x & 63] = 1;
}

// The boundary block of k_cont2 (kCont2Threads threads): thread t updates
// the coarse node t of the patch boundary lines (as the coarse level does;
// its new density also kept in LDS at that perimeter index) and the window
// part of the patch's boundary nodes t + q kCont2Threads, q < RF; after the
// barrier, their density from those coarse nodes (as the patch level
// interpolates it: r = 2 copy or mean, r = 4 linear along the line).  Every
// load of a thread comes before its stores.
constexpr int kCont2Threads = 1024;
template <int RF>
__device__ __forceinline__ void cont2_boundary(const ContArgs& C, const ContArgs& F) {
  __shared__ float sCn[kCont2Threads];
  const int t = threadIdx.x;
  const int nx = C.pR - C.pL + 1, ny = C.pT - C.pB - 1;  // x-lines, y-lines (inner)
  const int ncn = 2 * nx + 2 * (ny > 0 ? ny : 0);
  const int fx = F.R - F.L + 1, fy = F.T - F.B - 1;
  const int nfn = 2 * fx + 2 * (fy > 0 ? fy : 0);
  auto cnode = [&](int k, int& i, int& j) {
    if (k < 2 * nx) { i = C.pL + k % nx; j = k < nx ? C.pB : C.pT; }
    else { const int q = k - 2 * nx; i = q < ny ? C.pL : C.pR; j = C.pB + 1 + q % ny; }
  };
  auto fnode = [&](int k, int& i, int& j) {
    if (k < 2 * fx) { i = F.L + k % fx; j = k < fx ? F.B : F.T; }
    else { const int q = k - 2 * fx; i = q < fy ? F.L : F.R; j = F.B + 1 + q % fy; }
  };
  // perimeter index of coarse node (a, b) on a boundary line
  auto cidx = [&](int a, int b) {
    if (b == C.pB) return a - C.pL;
    if (b == C.pT) return nx + a - C.pL;
    return 2 * nx + (a == C.pL ? 0 : ny) + (b - C.pB - 1);
  };
  // loads: the coarse node's window, the patch nodes' windows, then the
  // coarse update (its density stencil)
  const bool hc = t < ncn;
  int ci = C.pL, cj = C.pB;
  if (hc) cnode(t, ci, cj);
  bool hf[RF];
  int fi[RF], fj[RF];
  size_t fo[RF];
  float fsv[RF], fe2[RF];
#pragma unroll
  for (int q = 0; q < RF; q++) {
    hf[q] = t + q * kCont2Threads < nfn;
    fi[q] = F.L; fj[q] = F.B;
    if (hf[q]) fnode(t + q * kCont2Threads, fi[q], fj[q]);
    fo[q] = (size_t)fj[q] * F.pitch + fi[q];
    fsv[q] = F.acc[fo[q]] * F.inv_spp;
    fe2[q] = 0.f;
  }
  const size_t co = (size_t)cj * C.pitch + ci;
  const float csv = C.acc[co] * C.inv_spp;
  float ce2 = 0.f;
  if (C.update) {
    for (int s = 0; s < kRing; s++) {
      ce2 += (s == C.slot) ? csv : C.ring[(size_t)s * C.plane + co];
#pragma unroll
      for (int q = 0; q < RF; q++) fe2[q] += (s == F.slot) ? fsv[q] : F.ring[(size_t)s * F.plane + fo[q]];
    }
  }
  float cnn = 0.f;
  if (C.update && hc) cnn = cont_update(C, co, ce2, ci > C.L, ci < C.R, cj > C.B, cj < C.T);
  // stores
  if (hc) {
    C.ring[(size_t)C.slot * C.plane + co] = csv;
    C.acc[co] = 0.f;
    if (C.update) {
      C.n1[co] = cnn;
      sCn[t] = cnn;
      if (!isfinite(cnn) || !isfinite(ce2)) C.err[t & 63] = 1;
    } else if (!isfinite(csv)) {
      C.err[t & 63] = 1;
    }
  }
#pragma unroll
  for (int q = 0; q < RF; q++) {
    if (!hf[q]) continue;
    F.ring[(size_t)F.slot * F.plane + fo[q]] = fsv[q];
    F.acc[fo[q]] = 0.f;
    if (C.update ? !isfinite(fe2[q]) : !isfinite(fsv[q])) F.err[t & 63] = 1;
  }
  __syncthreads();
  if (!F.update) return;
  auto interp = [&](int i, int j) {
    if constexpr (RF == 4) {
      const int a = i >> 2, b = j >> 2;
      const float ti = (i & 3) * 0.25f, tj = (j & 3) * 0.25f;
      const float c00 = sCn[cidx(a, b)];
      if ((i & 3) != 0) return (1.f - ti) * c00 + ti * sCn[cidx(a + 1, b)];
      if ((j & 3) != 0) return (1.f - tj) * c00 + tj * sCn[cidx(a, b + 1)];
      return c00;
    } else {
      const int a = i >> 1, b = j >> 1;
      if (((i | j) & 1) == 0) return sCn[cidx(a, b)];
      if (i & 1) return 0.5f * (sCn[cidx(a, b)] + sCn[cidx(a + 1, b)]);
      return 0.5f * (sCn[cidx(a, b)] + sCn[cidx(a, b + 1)]);
    }
  };
#pragma unroll
  for (int q = 0; q < RF; q++) {
    if (!hf[q]) continue;
    const float nn = interp(fi[q], fj[q]);
    F.n1[fo[q]] = nn;
    if (!isfinite(nn)) F.err[t & 63] = 1;
  }
}

// Continuity of both levels in one launch (rectangular patch, r = 2 or 4):
// blocks [0, ncb) the coarse level, [ncb, ncb + nfb) the patch, the last
// block the boundary lines.  Every node is updated by one thread; no block
// reads what another writes.
template <int RF>
__global__ __launch_bounds__(kCont2Threads) void k_cont2(ContArgs C, ContArgs F, int gxc, int ncb,
                                                         int gxf, int nfb) {
  const int b = blockIdx.x;
  if (b < ncb) cont_body<false, true, kCont2Threads>(C, b % gxc, b / gxc, C.slot, C.update);
  else if (b < ncb + nfb)
    cont_body<true, true, kCont2Threads>(F, (b - ncb) % gxf, (b - ncb) / gxf, F.slot, F.update);
  else cont2_boundary<RF>(C, F);
}

template <bool FINE>
__global__ __launch_bounds__(kThreads) void k_cont(ContArgs A) {
  cont_body<FINE>(A, blockIdx.x, blockIdx.y, A.slot, A.update);
}

template <bool FINE>
__global__ __launch_bounds__(kThreads) void k_cont_batch(const ContArgs* __restrict__ args,
                                                         const int2* __restrict__ blk,
                                                         int slot, int update) {
  const int2 bi = blk[blockIdx.x];
  const ContArgs& A = args[bi.x];
  cont_body<FINE>(A, bi.y % A.nbx, bi.y / A.nbx, slot, update);
}

// cell (i, j) of a fine level made of the active blocks of act
__device__ inline bool cell_active(const uint8_t* act, int fbs, int nbkx, int nbky, int i,
                                   int j) {
  if (i < 0 || j < 0) return false;
  const int bi = i >> fbs, bj = j >> fbs;
  return bi < nbkx && bj < nbky && act[(size_t)bj * nbkx + bi] != 0;
}

// Continuity on the fine level made of a union of blocks, over the listed
// 64 x TY node tiles: as for the patch, nodes with all four cells active are
// updated, the other nodes of the level (on the coarse/fine boundary) take
// the new coarse density, and coarse nodes whose four cells are active take
// the fine density at the coincident node (injection).  r = 2.
template <int TY>
__device__ __forceinline__ void cont_union_tile(const ContArgs& A, int2 t, int slot, int update) {
  const int i = t.x * kTX + (int)(threadIdx.x % kTX);
  for (int rr = threadIdx.x / kTX; rr < TY; rr += kThreads / kTX) {
    const int j = t.y * TY + rr;
    if (i > A.R || j > A.T) continue;
    const bool c00 = cell_active(A.act, A.fbs, A.nbkx, A.nbky, i - 1, j - 1);
    const bool c10 = cell_active(A.act, A.fbs, A.nbkx, A.nbky, i, j - 1);
    const bool c01 = cell_active(A.act, A.fbs, A.nbkx, A.nbky, i - 1, j);
    const bool c11 = cell_active(A.act, A.fbs, A.nbkx, A.nbky, i, j);
    if (!(c00 || c10 || c01 || c11)) continue;
    const size_t o = (size_t)j * A.pitch + i;
    const float sv = A.acc[o] * A.inv_spp;
    A.ring[(size_t)slot * A.plane + o] = sv;
    A.acc[o] = 0.f;
    if (!update) {
      if (!isfinite(sv)) A.err[threadIdx.x & 63] = 1;
      continue;
    }
    float e2 = 0.f;
    for (int s = 0; s < kRing; s++)
      e2 += (s == slot) ? sv : A.ring[(size_t)s * A.plane + o];
    float nn;
    if (!(c00 && c10 && c01 && c11)) {
      const int a = i >> 1, b = j >> 1, cp = A.cpitch;
      if (((i | j) & 1) == 0) nn = A.cn1[(size_t)b * cp + a];
      else if (i & 1) nn = 0.5f * (A.cn1[(size_t)b * cp + a] + A.cn1[(size_t)b * cp + a + 1]);
      else nn = 0.5f * (A.cn1[(size_t)b * cp + a] + A.cn1[(size_t)(b + 1) * cp + a]);
    } else {
      nn = cont_update(A, o, e2, true, true, true, true);
      if (((i | j) & 1) == 0) A.cn1[(size_t)(j >> 1) * A.cpitch + (i >> 1)] = nn;
    }
    A.n1[o] = nn;
    if (!isfinite(nn) || !isfinite(e2)) A.err[threadIdx.x & 63] = 1;
  }
}

template <int TY>
__global__ __launch_bounds__(kThreads) void k_cont_union(ContArgs A,
                                                         const int2* __restrict__ tiles) {
  cont_union_tile<TY>(A, tiles[blockIdx.x], A.slot, A.update);
}

template <int TY>
__global__ __launch_bounds__(kThreads) void k_cont_union_batch(const ContArgs* __restrict__ args,
                                                               const int2* __restrict__ blk,
                                                               int slot, int update) {
  const int2 bi = blk[blockIdx.x];
  const ContArgs& A = args[bi.x];
  cont_union_tile<TY>(A, A.utiles[bi.y], slot, update);
}

// ---------------------------------------------------------------------------
// Growth test, part 1: node flags (Sec. III.A threshold density, Sec. III.B
// gradient length) OR-reduced over each block.  Node (i, j) belongs to block
// (min(i/Bk, NBx-1), min(j/Bk, NBy-1)).  The decision is float32, without
// contraction, on n * 2^-60 (exact scaling keeping n^2 in range):
//   n > thr  or  (n > floor and gx*gx + gy*gy > g2 * (n*n)).
// ---------------------------------------------------------------------------
__device__ inline int node_flag(const FlagArgs &A, int i, int j) {
#pragma clang fp contract(off)
  const size_t o = (size_t)j * A.pitch + i;
  const float nv = A.n[o];
  if (nv > A.thr) return 1;
  if (!(nv > A.flo)) return 0;
  const float sc = 0x1p-60f;
  const float ns = nv * sc;
  float gx = 0.f, gy = 0.f;
  if (i > 0 && i < A.NX) gx = (A.n[o + 1] * sc - A.n[o - 1] * sc) * 0.5f;
  if (j > 0 && j < A.NY) gy = (A.n[o + A.pitch] * sc - A.n[o - A.pitch] * sc) * 0.5f;
  const float gx2 = gx * gx;
  const float gy2 = gy * gy;
  const float lhs = gx2 + gy2;
  const float n2 = ns * ns;
  const float rhs = A.g2 * n2;
  return lhs > rhs;
}

__global__ __launch_bounds__(256) void k_flag_blocks(FlagArgs A) {
  const int bx = blockIdx.x, by = blockIdx.y;
  const int ib = bx * A.Bk, jb = by * A.Bk;
  const int w = (bx == A.NBx - 1) ? A.NX + 1 - ib : A.Bk;
  const int h = (by == A.NBy - 1) ? A.NY + 1 - jb : A.Bk;
  int f = 0;
  for (int k = threadIdx.x; k < w * h; k += blockDim.x)
    f |= node_flag(A, ib + k % w, jb + k / w);
  f = __syncthreads_or(f);
  if (threadIdx.x == 0) A.bflag[by * A.NBx + bx] = (uint8_t)(f ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Growth test, part 2 (one block of 1024 threads): exclusive prefix sum of
// the block flags with wavefront shuffles, compaction of flagged block ids,
// bounding box, union with the current patch (growth only, Sec. III.D),
// clip to the margins, new extents into desc.
// desc: [0..3] current ext (blocks), [4..7] new ext (blocks), [8] count,
//       [9] changed, [10..13] margins xmin, ymin, xmax, ymax (blocks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan_bbox(ScanArgs A) {
  constexpr int NW = 1024 / 64;
  __shared__ int sTot[NW];
  __shared__ int sMin[2][NW], sMax[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry = 0;
  int mnx = 1 << 30, mny = 1 << 30, mxx = -1, mxy = -1;
  for (int base = 0; base < A.NB; base += 1024) {
    const int b = base + tid;
    const int f = (b < A.NB) ? (int)A.bflag[b] : 0;
    int x = f;  // inclusive scan within the wavefront
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) sTot[wv] = x;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NW; k++) {
      const int t = sTot[k];
      if (k < wv) before += t;
      total += t;
    }
    const int excl = carry + before + x - f;
    if (b < A.NB) {
      A.scan[b] = excl;
      if (f) {
        A.list[excl] = b;
        const int bx = b % A.NBx, by = b / A.NBx;
        mnx = min(mnx, bx); mny = min(mny, by);
        mxx = max(mxx, bx); mxy = max(mxy, by);
      }
    }
    carry += total;
    __syncthreads();
  }
  for (int d = 32; d >= 1; d >>= 1) {
    mnx = min(mnx, __shfl_xor(mnx, d, 64));
    mny = min(mny, __shfl_xor(mny, d, 64));
    mxx = max(mxx, __shfl_xor(mxx, d, 64));
    mxy = max(mxy, __shfl_xor(mxy, d, 64));
  }
  if (lane == 0) {
    sMin[0][wv] = mnx; sMin[1][wv] = mny;
    sMax[0][wv] = mxx; sMax[1][wv] = mxy;
  }
  __syncthreads();
  if (tid < 64) {
    int a = (lane < NW) ? sMin[0][lane] : (1 << 30);
    int c = (lane < NW) ? sMin[1][lane] : (1 << 30);
    int e = (lane < NW) ? sMax[0][lane] : -1;
    int g = (lane < NW) ? sMax[1][lane] : -1;
    for (int d = 32; d >= 1; d >>= 1) {
      a = min(a, __shfl_xor(a, d, 64));
      c = min(c, __shfl_xor(c, d, 64));
      e = max(e, __shfl_xor(e, d, 64));
      g = max(g, __shfl_xor(g, d, 64));
    }
    if (lane == 0) {
      int* D = A.desc;
      int x0 = a, y0 = c, x1 = e + 1, y1 = g + 1;
      if (carry == 0) { x0 = A.NBx; y0 = A.NBy; x1 = 0; y1 = 0; }
      if (D[2] > D[0]) {  // the patch only grows
        x0 = min(x0, D[0]); y0 = min(y0, D[1]);
        x1 = max(x1, D[2]); y1 = max(y1, D[3]);
      }
      x0 = max(x0, D[10]); y0 = max(y0, D[11]);
      x1 = min(x1, D[12]); y1 = min(y1, D[13]);
      if (x0 >= x1 || y0 >= y1) { x0 = y0 = x1 = y1 = 0; }
      D[4] = x0; D[5] = y0; D[6] = x1; D[7] = y1;
      D[8] = carry;
      D[9] = (x0 != D[0] || y0 != D[1] || x1 != D[2] || y1 != D[3]) ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Prolongation into the new part of the patch (Sec. III.D, Eq. (5a) area
// weights), one thread per fine node position of the new extents.  Entities
// that existed in the old patch keep their data.  E, J, n, window at the
// current coarse time; Hz at frac = 5/4 between coarse Hz^{n-1/2} and
// Hz^{n+1/2} (fine Hz lives at coarse n+3/4).  Positions are in quarter
// coarse units: fine index P -> 2P (on a coarse line) or 2P - 1 (a quarter
// below the next coarse half-point).
// ---------------------------------------------------------------------------
// Eq. (5a) at (U, V) / D in coarse index units (D = 2r: offsets 1/(2r))
__device__ inline float bilin4(const float* a, int pitch, int U4, int V4, int D = 4) {
  const int i = U4 / D, j = V4 / D;
  const float inv = D == 4 ? 0.25f : 0.125f;
  const float fu = (U4 % D) * inv, fv = (V4 % D) * inv;
  float v = 0.f;
  for (int di = 0; di < 2; di++) {
    const float wu = di ? fu : 1.f - fu;
    if (wu == 0.f) continue;
    for (int dj = 0; dj < 2; dj++) {
      const float wv = dj ? fv : 1.f - fv;
      if (wv == 0.f) continue;
      v += wu * wv * a[(size_t)(j + dj) * pitch + i + di];
    }
  }
  return v;
}

__global__ __launch_bounds__(kThreads) void k_prolong(ProlongArgs A) {
  const int i = A.L + blockIdx.x * kTX + (threadIdx.x % kTX);
  const int j = A.B + blockIdx.y * (kThreads / kTX) + (threadIdx.x / kTX);
  if (i > A.R || j > A.T) return;
  const size_t o = (size_t)j * A.pitch + i;
  const int cp = A.cpitch;
  const bool old = A.oR > A.oL;
  auto in_old = [&](int hx, int hy) {  // hx/hy: entity ends one short
    return old && i >= A.oL && i <= A.oR - hx && j >= A.oB && j <= A.oT - hy;
  };
  // positions in units of 1/(2r) coarse cells: a fine node i sits at 2i; a
  // fine half-offset entity at (i + 1/2)/r - 1/2 coarse half-offset
  // entities, i.e. at 2i + 1 - r
  const int D = A.rf == 4 ? 8 : 4, h = A.rf == 4 ? 3 : 1;
  // fine Hz after a coarse step sits at coarse n + 1 - 1/(2r): frac 3/2 - 1/(2r)
  const float fr = A.rf == 4 ? 1.375f : 1.25f;
  const float jsc = A.rf == 4 ? 0.25f : 0.5f;  // J~ scales with dt
  if (i < A.R && j < A.T && !in_old(1, 1)) {
    const float hp = bilin4(A.chz_prev, cp, 2 * i - h, 2 * j - h, D);
    const float hn = bilin4(A.chz, cp, 2 * i - h, 2 * j - h, D);
    A.hz[o] = (1.f - fr) * hp + fr * hn;
  }
  if (i < A.R && !in_old(1, 0)) {
    A.ex[o] = bilin4(A.cex, cp, 2 * i - h, 2 * j, D);
    A.jx[o] = jsc * bilin4(A.cjx, cp, 2 * i - h, 2 * j, D);
  }
  if (j < A.T && !in_old(0, 1)) {
    A.ey[o] = bilin4(A.cey, cp, 2 * i, 2 * j - h, D);
    A.jy[o] = jsc * bilin4(A.cjy, cp, 2 * i, 2 * j - h, D);
  }
  if (!in_old(0, 0)) {
    if (!A.keep_n) A.n[o] = bilin4(A.cn, cp, 2 * i, 2 * j, D);
    A.acc[o] = bilin4(A.cacc, cp, 2 * i, 2 * j, D);
    for (int s = 0; s < kRing; s++)
      A.ring[(size_t)s * A.plane + o] =
          bilin4(A.cring + (size_t)s * A.cplane, cp, 2 * i, 2 * j, D);
  }
}

// Prolongation into the blocks new to a union-of-blocks fine level (r = 2),
// over the listed 64 x TY tiles: every entity that belongs to the level now
// (act) and did not before (act_old) takes the Eq. (5a) values of k_prolong.
template <int TY>
__global__ __launch_bounds__(kThreads) void k_prolong_union(ProlongArgs A,
                                                            const int2* __restrict__ tiles) {
  const int2 t = tiles[blockIdx.x];
  const int i = t.x * kTX + (int)(threadIdx.x % kTX);
  const int cp = A.cpitch;
  auto now = [&](int a, int b) { return cell_active(A.act, A.fbs, A.nbkx, A.nbky, a, b); };
  auto was = [&](int a, int b) { return cell_active(A.act_old, A.fbs, A.nbkx, A.nbky, a, b); };
  for (int rr = threadIdx.x / kTX; rr < TY; rr += kThreads / kTX) {
    const int j = t.y * TY + rr;
    if (i > A.R || j > A.T) continue;
    const size_t o = (size_t)j * A.pitch + i;
    const bool n11 = now(i, j), n01 = now(i - 1, j), n10 = now(i, j - 1), n00 = now(i - 1, j - 1);
    const bool w11 = was(i, j), w01 = was(i - 1, j), w10 = was(i, j - 1), w00 = was(i - 1, j - 1);
    if (n11 && !w11) {
      const float hp = bilin4(A.chz_prev, cp, 2 * i - 1, 2 * j - 1);
      const float hn = bilin4(A.chz, cp, 2 * i - 1, 2 * j - 1);
      A.hz[o] = (1.f - 1.25f) * hp + 1.25f * hn;
    }
    if ((n11 || n10) && !(w11 || w10)) {
      A.ex[o] = bilin4(A.cex, cp, 2 * i - 1, 2 * j);
      A.jx[o] = 0.5f * bilin4(A.cjx, cp, 2 * i - 1, 2 * j);
    }
    if ((n11 || n01) && !(w11 || w01)) {
      A.ey[o] = bilin4(A.cey, cp, 2 * i, 2 * j - 1);
      A.jy[o] = 0.5f * bilin4(A.cjy, cp, 2 * i, 2 * j - 1);
    }
    if ((n11 || n01 || n10 || n00) && !(w11 || w01 || w10 || w00)) {
      A.n[o] = A.keep_n ? A.seed[o] : bilin4(A.cn, cp, 2 * i, 2 * j);
      A.acc[o] = bilin4(A.cacc, cp, 2 * i, 2 * j);
      for (int s = 0; s < kRing; s++)
        A.ring[(size_t)s * A.plane + o] = bilin4(A.cring + (size_t)s * A.cplane, cp, 2 * i, 2 * j);
    }
  }
}

// ---------------------------------------------------------------------------
// Pitched <-> dense copy with a scale factor (field read-out / write-in).
// ---------------------------------------------------------------------------
__global__ void k_gather(const float* src, int pitch, int i0, int j0, int cols,
                         int rows, float scale, float* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= cols || j >= rows) return;
  dst[(size_t)j * cols + i] = scale * src[(size_t)(j + j0) * pitch + i0 + i];
}

__global__ void k_scatter(const float* src, int cols, int rows, float scale,
                          float* dst, int pitch, int i0, int j0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= cols || j >= rows) return;
  dst[(size_t)(j + j0) * pitch + i0 + i] = scale * src[(size_t)j * cols + i];
}

// sum of the 8 ring planes (E_rms^2 read-out)
__global__ void k_ring_sum(const float* ring, size_t plane, int pitch, int i0,
                           int j0, int cols, int rows, float* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= cols || j >= rows) return;
  const size_t o = (size_t)(j + j0) * pitch + i0 + i;
  float s = 0.f;
  for (int k = 0; k < kRing; k++) s += ring[(size_t)k * plane + o];
  dst[(size_t)j * cols + i] = s;
}

// ---------------------------------------------------------------------------
// Base-level EM step, column-streaming form (Eqs. (1)-(3), Mur/PEC, TF/SF).
// One lane per node column: lanes 0-1 of each wavefront recompute the two
// columns left of the wave's 62 own columns, so x neighbours come from
// wavefront shuffles; the wave marches up a segment of rows keeping the
// previous row's new Hz / Ey / Ex in registers and the next two rows' loads
// in flight, so every plane is read once per row (a 1-row halo per segment,
// 2 of 64 columns per wave).  Own entities: Hz(i,j), Ex(i,j), Ey(i,j),
// node (i,j) for the own columns and the segment's rows.
// ---------------------------------------------------------------------------
struct RowData {
  float ex, ey, ey1, hz, jx, jy, n, n1, acc;
};

// Raw loads from clamped (always valid) addresses: nothing depends on the
// values until the row is consumed DEPTH rows later, so the loads stay in
// flight across iterations.
// Addressing of the streaming kernel: 32-bit byte offsets from the uniform
// plane bases (a plane is far below 4 GB; pitch * 4 < 2^24 is required by
// the parameter checks) save the per-lane 64-bit address arithmetic where
// the step is issue-bound (short segments, DEPTH 2, on grids too small to
// fill the chip); the long-segment form keeps 64-bit indices, which streamed
// faster (measured on 4096x2048 and 8192x4096).
#ifndef DMR_EM_O32
#define DMR_EM_O32(DEPTH) ((DEPTH) == 2)
#endif
struct RowAddr {
  size_t o64;
  unsigned o32;
};
__device__ __forceinline__ RowAddr row_addr(const EMArgs& A, int i, int j) {
  return RowAddr{(size_t)j * A.pitch + i,
                 __umul24((unsigned)j, (unsigned)A.pitch * 4u) + ((unsigned)i << 2)};
}
template <bool O32>
__device__ __forceinline__ float ldr(const float* p, const RowAddr& a) {
  if constexpr (O32) return ldo(p, a.o32);
  else return p[a.o64];
}
template <bool O32>
__device__ __forceinline__ void str(float* p, const RowAddr& a, float v) {
  if constexpr (O32) sto(p, a.o32, v);
  else p[a.o64] = v;
}

template <bool O32>
__device__ inline RowData load_row(const EMArgs& A, int i, int j) {
  RowData r;
  const int NX = A.R, NY = A.T;
  const int ic = min(max(i, 0), NX), jc = min(max(j, 0), NY);
  const int ic1 = min(max(i + 1, 0), NX);
  const RowAddr o = row_addr(A, ic, jc), o1 = row_addr(A, ic1, jc);
  r.ex = ldr<O32>(A.ex0, o); r.jx = ldr<O32>(A.jx0, o); r.ey = ldr<O32>(A.ey0, o);
  r.jy = ldr<O32>(A.jy0, o); r.ey1 = ldr<O32>(A.ey0, o1); r.hz = ldr<O32>(A.hz0, o);
  r.n = ldr<O32>(A.n, o); r.n1 = ldr<O32>(A.n, o1); r.acc = ldr<O32>(A.acc, o);
  return r;
}

// entries of row j that do not exist (outside the grid, or beyond the
// entity's own extent) read as zero
__device__ inline RowData mask_row(const EMArgs& A, const RowData& q, int i, int j) {
  const int NX = A.R, NY = A.T;
  const bool row_ok = j >= 0 && j <= NY;
  const bool exv = row_ok && i >= 0 && i < NX;
  const bool eyv = row_ok && j < NY && i >= 0 && i <= NX;
  const bool ey1v = row_ok && j < NY && i + 1 >= 0 && i + 1 <= NX;
  const bool ndv = row_ok && i >= 0 && i <= NX;
  const bool nd1v = row_ok && i + 1 >= 0 && i + 1 <= NX;
  RowData r;
  r.ex = exv ? q.ex : 0.f;
  r.jx = exv ? q.jx : 0.f;
  r.ey = eyv ? q.ey : 0.f;
  r.jy = eyv ? q.jy : 0.f;
  r.ey1 = ey1v ? q.ey1 : 0.f;
  r.hz = (eyv && i < NX) ? q.hz : 0.f;
  r.n = ndv ? q.n : 0.f;
  r.n1 = nd1v ? q.n1 : 0.f;
  r.acc = ndv ? q.acc : 0.f;
  return r;
}

template <int DEPTH, bool ST = false>
__device__ __forceinline__ void em_stream_body(const EMArgs& A, int cw, int k, int seg,
                                               int nseg, float ey_src, float hz_src) {
  constexpr bool O32 = DMR_EM_O32(DEPTH);
  const int NX = A.R, NY = A.T;
  const int lane = threadIdx.x & 63;
  const int c0 = cw * 62;  // first own column of this wave
  const int i = c0 - 2 + lane;
  const bool own = lane >= 2 && i <= NX;
  const int j0 = k * seg;
  const int j1 = (k == nseg - 1) ? NY + 1 : j0 + seg;
  const bool wave_has_left = c0 - 2 <= 0 && 0 <= c0 + 61;   // column 0 in the wave
  const bool wave_has_right = c0 - 2 <= NX && NX <= c0 + 61;
  const bool exv = i >= 0 && i < NX;
  const bool eyc = i >= 0 && i <= NX;
  const float S = A.S, c1 = A.c1, a = A.a, kn = A.kn, cm = A.cmur;
  // combined step: the coarse entities strictly inside the patch are written
  // by the patch tiles' fine -> coarse transfer in the same launch
  const bool skc = A.skip_on && i >= A.sL && i < A.sR;  // cells, x-edges
  const bool sky = A.skip_on && i > A.sL && i < A.sR;   // y-edges
  const bool mur_x = A.bc_x == kBcMur, mur_y = A.bc_y == kBcMur;

  const int js = j0 > 0 ? j0 - 1 : 0;
  // rows js .. js+DEPTH in flight; buf[0] is the current row
  RowData buf[DEPTH + 1];
#pragma unroll
  for (int d = 0; d <= DEPTH; d++) buf[d] = load_row<O32>(A, i, min(js + d, j1));
  float hzn_p = 0.f, eyn_p = 0.f, exn_p = 0.f, exo_p = 0.f;
  // row-0 Mur edge Ex(i,0) waits for Ex(i,1): its old value, current, density
  float ex0_old = 0.f, jx0_old = 0.f, kap0 = 0.f, acc0 = 0.f;

  // one row of the segment; rc/rn: raw rows j and j+1
  auto row = [&](int j, const RowData& rc, const RowData& rn) {
    const RowData cur = mask_row(A, rc, i, j);
    const RowData nxt = mask_row(A, rn, i, j + 1);
    const bool store = j >= j0 && j < j1;
    const RowAddr o = row_addr(A, i, j);  // used only where (i, j) is stored (exists)
    if (ST && store && own) {  // replay: the values entering the step
      if (exv) str<O32>(A.stix, o, cur.ex);
      if (eyc && j < NY) str<O32>(A.stiy, o, cur.ey);
      if (eyc) str<O32>(A.stn, o, cur.n);
    }

    // Faraday, Eq. (2)
    float hzn = 0.f;
    if (exv && j < NY) {
      hzn = base_hz(cur.hz, S, cur.ey1, cur.ey, nxt.ex, cur.ex);
      if (i == A.is - 1) hzn += S * ey_src;
      if (store && own && !(skc && j >= A.sB && j < A.sT)) str<O32>(A.hz1, o, hzn);
    }
    const float hzl = __shfl_up(hzn, 1, 64);  // Hz(i-1, j)

    // Ampere + Drude, Eqs. (1), (3): x-edges
    float exn = 0.f;
    const float kapx = base_kap(kn, cur.n, cur.n1);
    if (exv) {
      if (j > 0 && j < NY) {
        exn = base_ex(cur.ex, kapx, S, hzn, hzn_p, c1, cur.jx);
        if (ST && store && own) str<O32>(A.stox, o, exn);
        if (store && own && !(skc && j > A.sB && j < A.sT)) {
          str<O32>(A.ex1, o, exn);
          str<O32>(A.jx1, o, a * cur.jx + 2.f * kapx * (cur.ex + exn));
        }
      } else if (j == NY) {
        exn = mur_y ? exo_p + cm * (exn_p - cur.ex) : 0.f;
        if (ST && store && own) str<O32>(A.stox, o, exn);
        if (store && own) {
          str<O32>(A.ex1, o, exn);
          str<O32>(A.jx1, o, a * cur.jx + 2.f * kapx * (cur.ex + exn));
        }
      } else if (j == 0) {  // finished with row 1
        ex0_old = cur.ex;
        jx0_old = cur.jx;
        kap0 = kapx;
      }
    }
    // y-edges
    float eyn = 0.f;
    const float kapy = base_kap(kn, cur.n, nxt.n);
    if (eyc && j < NY && i > 0 && i < NX) {
      float curl = -S * (hzn - hzl);
      if (i == A.is) curl += S * hz_src;
      eyn = base_ey(cur.ey, kapy, curl, c1, cur.jy);
    }
    if (j < NY && (wave_has_left || wave_has_right)) {
      const float nr = __shfl_down(eyn, 1, 64), orr = __shfl_down(cur.ey, 1, 64);
      const float nl = __shfl_up(eyn, 1, 64), ol = __shfl_up(cur.ey, 1, 64);
      if (i == 0) eyn = mur_x ? orr + cm * (nr - cur.ey) : 0.f;
      if (i == NX) eyn = mur_x ? ol + cm * (nl - cur.ey) : 0.f;
    }
    if (ST && eyc && j < NY && store && own) str<O32>(A.stoy, o, eyn);
    if (eyc && j < NY && store && own && !(sky && j >= A.sB && j < A.sT)) {
      str<O32>(A.ey1, o, eyn);
      str<O32>(A.jy1, o, a * cur.jy + 2.f * kapy * (cur.ey + eyn));
    }

    // deferred bottom row: Mur edge Ex(i,0) and the window at node row 0
    if (j == 1 && j0 == 0) {
      float ex0 = 0.f;
      if (exv) {
        ex0 = mur_y ? cur.ex + cm * (exn - ex0_old) : 0.f;
        if (own) {
          if (ST) str<O32>(A.stox, row_addr(A, i, 0), ex0);
          str<O32>(A.ex1, row_addr(A, i, 0), ex0);
          str<O32>(A.jx1, row_addr(A, i, 0), a * jx0_old + 2.f * kap0 * (ex0_old + ex0));
        }
      }
      const float exl0 = __shfl_up(ex0, 1, 64);
      if (own && eyc) {
        float sx = 0.f, e2;
        int cx = 0;
        if (i > 0) { sx += exl0 * exl0; cx++; }
        if (i < NX) { sx += ex0 * ex0; cx++; }
        e2 = (cx == 2 ? 0.5f * sx : sx) + eyn_p * eyn_p;
        str<O32>(A.acc, row_addr(A, i, 0), acc0 + e2);
      }
    }
    // window at node (i, j)
    const float exl = __shfl_up(exn, 1, 64);
    if (j > 0) {
      if (store && own) {
        float sx = 0.f, sy = 0.f;
        int cx = 0, cy = 0;
        if (i > 0) { sx += exl * exl; cx++; }
        if (i < NX) { sx += exn * exn; cx++; }
        sy += eyn_p * eyn_p; cy++;
        if (j < NY) { sy += eyn * eyn; cy++; }
        const float e2 = (cx == 2 ? 0.5f * sx : sx) + (cy == 2 ? 0.5f * sy : sy);
        str<O32>(A.acc, o, cur.acc + e2);
      }
    } else {
      acc0 = cur.acc;
    }
    hzn_p = hzn;
    eyn_p = eyn;
    exn_p = exn;
    exo_p = cur.ex;
  };
  // unrolled by DEPTH+1 so the pipeline slots rotate by index: slot u holds
  // row jb+u until it is consumed, then takes row jb+u+DEPTH+1
  // the loads stay unconditional (rows past the segment are computed
  // from clamped reads and not stored), so the wait for a slot's loads is
  // exact rather than a drain of everything in flight
  // A wave whose columns and rows are all interior (no outer boundary, no
  // source column, no patch region, rows 1 .. NY-1 with the next row inside)
  // takes the same arithmetic without the tests for those cases: every
  // condition the general row tests holds there, and each value is formed
  // by the same expressions.  Short segments only, where the step is
  // issue-bound (measured: no gain on the long-segment, bandwidth-bound form)
  constexpr bool FAST = !ST && DEPTH == 2;
  auto row_fast = [&](int j, const RowData& cur, const RowData& nxt) {
    const bool store = j >= j0 && j < j1;
    const RowAddr o = row_addr(A, i, j);
    const float hzn = base_hz(cur.hz, S, cur.ey1, cur.ey, nxt.ex, cur.ex);
    if (store && own) str<O32>(A.hz1, o, hzn);
    const float hzl = __shfl_up(hzn, 1, 64);
    const float kapx = base_kap(kn, cur.n, cur.n1);
    const float exn = base_ex(cur.ex, kapx, S, hzn, hzn_p, c1, cur.jx);
    if (store && own) {
      str<O32>(A.ex1, o, exn);
      str<O32>(A.jx1, o, a * cur.jx + 2.f * kapx * (cur.ex + exn));
    }
    const float kapy = base_kap(kn, cur.n, nxt.n);
    const float curl = -S * (hzn - hzl);
    const float eyn = base_ey(cur.ey, kapy, curl, c1, cur.jy);
    if (store && own) {
      str<O32>(A.ey1, o, eyn);
      str<O32>(A.jy1, o, a * cur.jy + 2.f * kapy * (cur.ey + eyn));
    }
    const float exl = __shfl_up(exn, 1, 64);
    if (store && own) {
      float sx = 0.f, sy = 0.f;
      sx += exl * exl;
      sx += exn * exn;
      sy += eyn_p * eyn_p;
      sy += eyn * eyn;
      const float hx = 0.5f * sx;
      const float hy = 0.5f * sy;
      const float e2 = hx + hy;
      str<O32>(A.acc, o, cur.acc + e2);
    }
    hzn_p = hzn;
    eyn_p = eyn;
  };
  const bool col_in = c0 - 2 >= 1 && c0 + 61 <= NX - 1;
  const bool no_src = A.is <= 0 || A.is < c0 - 2 || A.is - 1 > c0 + 61;
  const bool no_skip = !A.skip_on || A.sR < c0 - 2 || A.sL > c0 + 61 || A.sT < js || A.sB > j1;
  const bool fast = FAST && col_in && no_src && no_skip && js >= 1 && j1 <= NY - 1;
  auto run = [&](auto&& rowf) {
    for (int jb = js; jb < j1; jb += DEPTH + 1) {
#pragma unroll
      for (int u = 0; u <= DEPTH; u++) {
        const int j = jb + u;
        rowf(j, buf[u], buf[u == DEPTH ? 0 : u + 1]);
        // rows past j1 are not needed: re-read row j1 (a cache hit)
        buf[u] = load_row<O32>(A, i, min(j + DEPTH + 1, j1));
      }
    }
  };
  if constexpr (FAST) {
    if (fast) run(row_fast);
    else run(row);
  } else {
    run(row);
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each
// XCD has its own L2.  Hand XCD x a contiguous band of the row-major
// (column block, segment) grid so that neighbouring blocks, which read the
// same cache lines at their common columns and rows, share an L2.
__device__ inline int xcd_band(int L, int N) {
  const int x = L & 7, k = L >> 3, q = N >> 3, r = N & 7;
  return x * q + min(x, r) + k;
}

template <int DEPTH, bool ST = false>
__global__ __launch_bounds__(kThreads) void k_em_stream(EMArgs A, int seg, int nseg, int nbx) {
  const int b = xcd_band(blockIdx.x, nbx * nseg);
  em_stream_body<DEPTH, ST>(A, (b % nbx) * (kThreads / 64) + (threadIdx.x >> 6), b / nbx, seg, nseg,
                        A.ey_src, A.hz_src);
}

// batched form; the incident values of step k of the current interval come
// from src[instance * kSrcSteps + k]
template <int DEPTH>
__global__ __launch_bounds__(kThreads) void k_em_stream_batch(const EMArgs* __restrict__ args,
                                                              const int2* __restrict__ blk,
                                                              const float2* __restrict__ src,
                                                              int k) {
  const int2 bi = blk[blockIdx.x];
  const EMArgs& A = args[bi.x];
  const float2 sv = src[(size_t)bi.x * kSrcSteps + k];
  em_stream_body<DEPTH>(A, (bi.y % A.nbx) * (kThreads / 64) + (threadIdx.x >> 6), bi.y / A.nbx,
                        A.seg, A.nseg, sv.x, sv.y);
}

// ---------------------------------------------------------------------------
// One patch substep (rectangle, r = 2) in streaming form, for patches too
// large for the tile kernels to reach the memory rate: a wave owns 58 node
// columns (lanes 3..60, three halo lanes on each side for the filter's and
// Faraday's x-neighbours, taken by wave shuffles) and walks a segment of rows
// upward.  The filter's vertical window lives in registers: raw E of rows
// j+1..j+3, its Laplacian of rows j..j+2, the filtered E of rows j, j+1; the
// other inputs of a row are consumed three rows after their load.  Each
// entity is computed with the same helpers and operands as by fine_tile, so
// the results are identical; the fine -> coarse transfer of the last
// substep is taken row by row (Hz and Ey of node row j when row j+1 is done).
// ---------------------------------------------------------------------------
struct FRow {
  float ex, ey;                  // raw E of row j + 2 of the slot's row j
  float hz, jx, jy, n, acc;      // row j
  float bo0, bo1, bn0, bn1;      // coarse Ey of row j's Eq. (5b) value (old / new)
};

// raw loads from clamped (always valid) addresses: E of fine row je, the
// other inputs of row jf; the Eq. (5b) inputs are those of the patch side
// nearer to the column
__device__ __forceinline__ FRow fine_row(const EMArgs& A, int i, int je, int jf) {
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const int ic = min(max(i, L), R);
  const size_t oe = (size_t)min(max(je, B), T) * A.pitch + ic;
  const size_t of = (size_t)min(max(jf, B), T) * A.pitch + ic;
  FRow r;
  r.ex = A.ex0[oe]; r.ey = A.ey0[oe];
  r.hz = A.hz0[of]; r.jx = A.jx0[of]; r.jy = A.jy0[of]; r.n = A.n[of]; r.acc = A.acc[of];
  // Ey on side column L or R at fine row jb: coarse edges (I, c), (I, c + 1)
  const int jb = min(max(jf, B), T - 1);
  const int I = (2 * i <= L + R ? L : R) >> 1;
  const int c = (jb & 1) ? (jb >> 1) : (jb >> 1) - 1;
  const size_t b0 = (size_t)c * A.cpitch + I;
  r.bo0 = A.cey0[b0]; r.bo1 = A.cey0[b0 + A.cpitch];
  r.bn0 = A.cey1[b0]; r.bn1 = A.cey1[b0 + A.cpitch];
  return r;
}

template <int DEPTH>
__device__ __forceinline__ void fine_stream_body(const EMArgs& A, int cw, int k, int seg,
                                                 int nseg) {
  const int L = A.L, R = A.R, B = A.B, T = A.T;
  const int lane = threadIdx.x & 63;
  const int i = L + cw * 58 - 3 + lane;
  const bool own = lane >= 3 && lane <= 60 && i <= R;
  const int j0 = B + k * seg;
  const int j1 = (k == nseg - 1) ? T + 1 : j0 + seg;
  const bool filt = A.gamma > 0.f;
  const float S = A.S, c1 = A.c1, a = A.a, kn = A.kn, gam = A.gamma, frac = A.frac;
  const bool cx_ = i >= L && i < R;   // x-edge / cell column
  const bool cy_ = i >= L && i <= R;  // y-edge / node column
  auto ex_ok = [&](int ii, int jj) { return ii >= L && ii < R && jj >= B && jj <= T; };
  auto ey_ok = [&](int ii, int jj) { return ii >= L && ii <= R && jj >= B && jj < T; };
  auto nd_ok = [&](int jj) { return cy_ && jj >= B && jj <= T; };
  // Eq. (5b) Ex values of the bottom and top rows (space weights by column)
  float exB = 0.f, exT = 0.f;
  {
    const int ib = min(max(i, L), R - 1);
    const int ic = (ib & 1) ? (ib >> 1) : (ib >> 1) - 1;
    const float w0 = (ib & 1) ? 0.75f : 0.25f, w1 = (ib & 1) ? 0.25f : 0.75f;
    const size_t oB = (size_t)(B >> 1) * A.cpitch + ic, oT = (size_t)(T >> 1) * A.cpitch + ic;
    exB = cfb(w0, w1, A.cex0[oB], A.cex0[oB + 1], A.cex1[oB], A.cex1[oB + 1], frac);
    exT = cfb(w0, w1, A.cex0[oT], A.cex0[oT + 1], A.cex1[oT], A.cex1[oT + 1], frac);
  }

  // raw E masked to the patch (zero elsewhere, as fine_tile's LDS copy)
  auto mx = [&](float v, int jj) { return ex_ok(i, jj) ? v : 0.f; };
  auto my = [&](float v, int jj) { return ey_ok(i, jj) ? v : 0.f; };
  // Laplacian of row jj from raw rows jj-1 (d), jj (c), jj+1 (u)
  auto lapx = [&](float d, float c, float u, int jj) {
    const float l = __shfl_up(c, 1, 64), r = __shfl_down(c, 1, 64);
    if (!ex_ok(i, jj)) return 0.f;
    return lap5(c, ex_ok(i - 1, jj) ? l : c, ex_ok(i + 1, jj) ? r : c,
                ex_ok(i, jj - 1) ? d : c, ex_ok(i, jj + 1) ? u : c);
  };
  auto lapy = [&](float d, float c, float u, int jj) {
    const float l = __shfl_up(c, 1, 64), r = __shfl_down(c, 1, 64);
    if (!ey_ok(i, jj)) return 0.f;
    return lap5(c, ey_ok(i - 1, jj) ? l : c, ey_ok(i + 1, jj) ? r : c,
                ey_ok(i, jj - 1) ? d : c, ey_ok(i, jj + 1) ? u : c);
  };
  // filtered E of row jj from its raw value and the Laplacian rows jj-1..jj+1
  auto filx = [&](float raw, float qd, float qc, float qu, int jj) {
    const float l = __shfl_up(qc, 1, 64), r = __shfl_down(qc, 1, 64);
    if (!ex_ok(i, jj)) return 0.f;
    if (!filt || jj == B || jj == T) return raw;
    const float l2 = lap5(qc, ex_ok(i - 1, jj) ? l : qc, ex_ok(i + 1, jj) ? r : qc,
                          ex_ok(i, jj - 1) ? qd : qc, ex_ok(i, jj + 1) ? qu : qc);
    return filter_e(raw, gam, l2);
  };
  auto fily = [&](float raw, float qd, float qc, float qu, int jj) {
    const float l = __shfl_up(qc, 1, 64), r = __shfl_down(qc, 1, 64);
    if (!ey_ok(i, jj)) return 0.f;
    if (!filt || i == L || i == R) return raw;
    const float l2 = lap5(qc, ey_ok(i - 1, jj) ? l : qc, ey_ok(i + 1, jj) ? r : qc,
                          ey_ok(i, jj - 1) ? qd : qc, ey_ok(i, jj + 1) ? qu : qc);
    return filter_e(raw, gam, l2);
  };

  const int js = j0 > B ? j0 - 1 : j0;
  // warm-up: raw E of rows js-2 .. js+2 (Laplacian rows js-1 .. js+1,
  // filtered row js) and the other inputs of row js
  float ax[5], ay[5];
  FRow D0 = fine_row(A, i, js - 2, js);
  ax[0] = D0.ex; ay[0] = D0.ey;
#pragma unroll
  for (int d = 1; d < 5; d++) {
    const int jj = min(max(js - 2 + d, B), T);
    const size_t oe = (size_t)jj * A.pitch + min(max(i, L), R);
    ax[d] = A.ex0[oe];
    ay[d] = A.ey0[oe];
  }
  float rx1, rx2, ry1, ry2, qx0, qx1, qy0, qy1, fx0, fy0;
  {
#pragma unroll
    for (int d = 0; d < 5; d++) { ax[d] = mx(ax[d], js - 2 + d); ay[d] = my(ay[d], js - 2 + d); }
    const float qxm = lapx(ax[0], ax[1], ax[2], js - 1), qym = lapy(ay[0], ay[1], ay[2], js - 1);
    qx0 = lapx(ax[1], ax[2], ax[3], js); qy0 = lapy(ay[1], ay[2], ay[3], js);
    qx1 = lapx(ax[2], ax[3], ax[4], js + 1); qy1 = lapy(ay[2], ay[3], ay[4], js + 1);
    fx0 = filx(ax[2], qxm, qx0, qx1, js);
    fy0 = fily(ay[2], qym, qy0, qy1, js);
    rx1 = ax[3]; rx2 = ax[4]; ry1 = ay[3]; ry2 = ay[4];
  }
  // slot of iteration j: raw E of row j+3, the other inputs of row j+1;
  // slots of iterations js .. js+DEPTH in flight, buf[0] the next to arrive
  FRow buf[DEPTH + 1];
#pragma unroll
  for (int d = 0; d <= DEPTH; d++)
    buf[d] = fine_row(A, i, min(js + d + 3, j1 + 2), min(js + d + 1, j1));
  // the previous row: new / old Hz, new Ey and Jy (Ampere, window, transfer)
  float hn_p = 0.f, ho_p = 0.f, eyn_p = 0.f, jyn_p = 0.f;

  auto row = [&](int j, const FRow& nw) {
    const bool store = j >= j0 && j < j1;
    const size_t o = (size_t)j * A.pitch + i;
    // Laplacian row j+2, filtered row j+1
    const float rx3 = mx(nw.ex, j + 3), ry3 = my(nw.ey, j + 3);
    const float qx2 = lapx(rx1, rx2, rx3, j + 2), qy2 = lapy(ry1, ry2, ry3, j + 2);
    const float fx1 = filx(rx1, qx0, qx1, qx2, j + 1);
    const float fy1 = fily(ry1, qy0, qy1, qy2, j + 1);
    // Faraday, Eq. (2)
    const float fyr = __shfl_down(fy0, 1, 64);
    float h = 0.f, ho = 0.f;
    if (cx_ && j >= B && j < T) {
      ho = D0.hz;
      h = faraday(ho, S, fyr - fy0, fx1 - fx0);
      if (store && own) A.hz1[o] = h;
    }
    const float hl = __shfl_up(h, 1, 64);
    // densities at the edges' end nodes (zero outside the patch)
    const float n0 = nd_ok(j) ? D0.n : 0.f, n1 = nd_ok(j + 1) ? nw.n : 0.f;
    const float n0r = __shfl_down(n0, 1, 64);
    // Ampere + Drude, Eqs. (1), (3); Eq. (5b) on the boundary
    float exn = 0.f, jxn = 0.f;
    if (ex_ok(i, j)) {
      const float e = fx0;
      const float ne = 0.5f * (n0 + n0r);
      const float kap = kn * ne;
      const float jo = D0.jx;
      if (j != B && j != T) {
        const float dh = h - hn_p;
        exn = ampere(e, kap, S * dh, c1, jo);
      } else {
        exn = j == B ? exB : exT;
      }
      jxn = drude(a, jo, kap, e, exn);
      if (store && own) { A.ex1[o] = exn; A.jx1[o] = jxn; }
    }
    float eyn = 0.f, jyn = 0.f;
    if (ey_ok(i, j)) {
      const float e = fy0;
      const float ne = 0.5f * (n0 + n1);
      const float kap = kn * ne;
      const float jo = D0.jy;
      if (i != L && i != R) {
        const float dh = h - hl;
        eyn = ampere(e, kap, -S * dh, c1, jo);
      } else {
        const float w0 = (j & 1) ? 0.75f : 0.25f, w1 = (j & 1) ? 0.25f : 0.75f;
        eyn = cfb(w0, w1, D0.bo0, D0.bo1, D0.bn0, D0.bn1, frac);
      }
      jyn = drude(a, jo, kap, e, eyn);
      if (store && own) { A.ey1[o] = eyn; A.jy1[o] = jyn; }
    }
    // window at node (i, j)
    const float exl = __shfl_up(exn, 1, 64);
    if (store && own && nd_ok(j)) {
      float sx = 0.f, sy = 0.f;
      int cx = 0, cy = 0;
      if (i > L) { const float v = exl; sx += v * v; cx++; }
      if (i < R) { const float v = exn; sx += v * v; cx++; }
      if (j > B) { const float v = eyn_p; sy += v * v; cy++; }
      if (j < T) { const float v = eyn; sy += v * v; cy++; }
      const float e2 = win_e2(sx, cx, sy, cy);
      A.acc[o] = D0.acc + e2;
    }
    // fine -> coarse transfer (coarse entities strictly inside the patch)
    const float exr = __shfl_down(exn, 1, 64), jxr = __shfl_down(jxn, 1, 64);
    const float hr = __shfl_down(h, 1, 64), hor = __shfl_down(ho, 1, 64);
    const float hr_p = __shfl_down(hn_p, 1, 64), hor_p = __shfl_down(ho_p, 1, 64);
    if (A.restrict_on && own && ((i - L) & 1) == 0) {
      // x-edges of node row j
      if (store && ((j - B) & 1) == 0 && ex_ok(i, j) && j != B && j != T) {
        const size_t co = (size_t)(j >> 1) * A.cpitch + (i >> 1);
        A.cex[co] = 0.5f * (exn + exr);
        A.cjx[co] = jxn + jxr;  // J~ scales with dt
      }
      // cells and y-edges of node row j - 1 (rows j - 1 and j are done)
      const int jn = j - 1;
      if (jn >= j0 && jn < j1 && ((jn - B) & 1) == 0) {
        const size_t co = (size_t)(jn >> 1) * A.cpitch + (i >> 1);
        if (cx_ && jn >= B && jn < T) {
          float s = 0.f;
          s += 0.5f * (ho_p + hn_p);
          s += 0.5f * (ho + h);
          s += 0.5f * (hor_p + hr_p);
          s += 0.5f * (hor + hr);
          A.chz[co] = 0.25f * s;
        }
        if (ey_ok(i, jn) && i != L && i != R) {
          A.cey[co] = 0.5f * (eyn_p + eyn);
          A.cjy[co] = jyn_p + jyn;
        }
      }
    }
    // rotate the row windows
    rx1 = rx2; rx2 = rx3; ry1 = ry2; ry2 = ry3;
    qx0 = qx1; qx1 = qx2; qy0 = qy1; qy1 = qy2;
    fx0 = fx1; fy0 = fy1;
    D0 = nw;
    hn_p = h; ho_p = ho; eyn_p = eyn; jyn_p = jyn;
  };
  // unrolled by DEPTH+1 so the pipeline slots rotate by index (as in
  // em_stream_body); rows past the segment are computed from clamped reads
  // and not stored, so every iteration issues the same memory operations
  // and the wait for a slot's loads is exact
  for (int jb = js; jb < j1; jb += DEPTH + 1) {
#pragma unroll
    for (int u = 0; u <= DEPTH; u++) {
      const int j = jb + u;
      row(j, buf[u]);
      const int jn = j + DEPTH + 1;  // the iteration this slot serves next
      buf[u] = fine_row(A, i, min(jn + 3, j1 + 2), min(jn + 1, j1));
    }
  }
}

template <int DEPTH>
__global__ __launch_bounds__(kThreads) void k_fine_stream(EMArgs A, int seg, int nseg, int nbx) {
  const int b = xcd_band(blockIdx.x, nbx * nseg);
  fine_stream_body<DEPTH>(A, (b % nbx) * (kThreads / 64) + (threadIdx.x >> 6), b / nbx, seg,
                          nseg);
}

// ---------------------------------------------------------------------------
// Combined step: the base-level EM step and both patch substeps of a coarse
// step in one launch.  The first blocks are TW x TY patch tiles, the last ncb
// are base-level waves (16 per block, column-wave w % waves_x of segment
// w / waves_x, blocks banded over the XCDs).  The tiles compute the coarse E
// after the step on their boundary lines themselves.  The base waves do not store
// the coarse entities the tiles' fine -> coarse transfer writes.
// ---------------------------------------------------------------------------
// R4: refinement factor 4, the launch runs the base step and the first pair
// of the four substeps (the second pair, with the fine -> coarse transfer,
// is a k_fine2_fast launch of its own)
template <int DEPTH, int TY, bool ST = false, int TW = kTX, bool R4 = false>
__global__ __launch_bounds__(step_threads(ST, TY)) void k_dmr_step(EMArgs C, EMArgs F, int seg,
                                                                       int nseg, int waves_x,
                                                                       int ncb, int nbx_f) {
  constexpr int NTC = step_threads(ST, TY);
  // the patch tiles are the longer chain: they take the first blocks, which
  // the dispatcher starts first
  const int ntl = gridDim.x - ncb;
  const int b = blockIdx.x;
  if (b >= ntl) {
    const int w = xcd_band(b - ntl, ncb) * (NTC / 64) + (threadIdx.x >> 6);
    const int k = w / waves_x;
    if (k < nseg) em_stream_body<DEPTH, ST>(C, w % waves_x, k, seg, nseg, C.ey_src, C.hz_src);
    return;
  }
  if constexpr (!ST && TY == 4)
    fine2_fast<TY, NTC, TW, R4>(F, b % nbx_f, b / nbx_f, F.cey_src, F.chz_src);
  else
    fine2_tile<TY, NTC, true, ST, R4, TW>(F, b % nbx_f, b / nbx_f, F.cey_src, F.chz_src);
}

// Batched combined step: blk[b] = (instance, g), g >= 0 a group of 16 base
// waves of the instance (column wave w % waves_x of segment w / waves_x),
// g < 0 its patch tile -1 - g (64 x TY).  The incident values of step k of
// the interval come from src, as in k_em_stream_batch.
template <int DEPTH, int TY>
__global__ __launch_bounds__(kFineThreads) void k_dmr_step_batch(const EMArgs* __restrict__ cargs,
                                                                 const EMArgs* __restrict__ fargs,
                                                                 const int2* __restrict__ blk,
                                                                 const float2* __restrict__ src,
                                                                 int k) {
  const int2 bi = blk[blockIdx.x];
  const float2 sv = src[(size_t)bi.x * kSrcSteps + k];
  if (bi.y >= 0) {
    const EMArgs& C = cargs[bi.x];
    const int waves_x = C.nbx * (kThreads / 64);
    const int w = bi.y * (kFineThreads / 64) + (threadIdx.x >> 6);
    const int sg = w / waves_x;
    if (sg < C.nseg) em_stream_body<DEPTH>(C, w % waves_x, sg, C.seg, C.nseg, sv.x, sv.y);
    return;
  }
  const EMArgs& F = fargs[bi.x];
  const int t = -1 - bi.y;
  fine2_tile<TY, kFineThreads, true, false, false, kTX>(F, t % F.nbx, t / F.nbx, sv.x, sv.y);
}

// ---- host-side launchers ----------------------------------------------------
// patch kernels: 64 x TY node tiles, NT threads per tile
#define DMR_LAUNCH_TILE(KERNEL, TY_, nt, A, st)                                          \
  do {                                                                                  \
    const dim3 g_((A.R - A.L + 1 + kTX - 1) / kTX, (A.T - A.B + 1 + (TY_)-1) / (TY_));  \
    if ((nt) >= 1024) hipLaunchKernelGGL((KERNEL<TY_, 1024>), g_, dim3(1024), 0, st, A); \
    else hipLaunchKernelGGL((KERNEL<TY_, 256>), g_, dim3(256), 0, st, A);                \
  } while (0)
// the replay form (stores for the adjoint), 1024 threads
#define DMR_LAUNCH_TILE_ST(KERNEL, TY_, A, st)                                           \
  do {                                                                                  \
    const dim3 g_((A.R - A.L + 1 + kTX - 1) / kTX, (A.T - A.B + 1 + (TY_)-1) / (TY_));  \
    hipLaunchKernelGGL((KERNEL<TY_, 1024, true>), g_, dim3(1024), 0, st, A);             \
  } while (0)

hipError_t launch_em(const EMArgs& A, bool fine, int ty, int nt, hipStream_t st) {
  if (!fine) return hipErrorInvalidValue;  // the base level uses the streaming kernel
  switch (ty) {
  case 4: DMR_LAUNCH_TILE(k_fine, 4, nt, A, st); break;
  case 8: DMR_LAUNCH_TILE(k_fine, 8, nt, A, st); break;
  default: DMR_LAUNCH_TILE(k_fine, 16, nt, A, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_fine_stream(const EMArgs& A, int seg, int depth, hipStream_t st) {
  if (A.rf == 4 || A.act || A.hz_save || A.hz_lo || A.stn) return hipErrorInvalidValue;
  seg = seg < 2 ? 2 : (seg & ~1);  // segments start at even offsets from B
  const int waves = (A.R - A.L + 1 + 57) / 58;
  const int nbx = (waves + kThreads / 64 - 1) / (kThreads / 64);
  const int nseg = (A.T - A.B + 1 + seg - 1) / seg;
  const dim3 g(nbx * nseg);
  if (depth >= 4) hipLaunchKernelGGL(k_fine_stream<4>, g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
  else hipLaunchKernelGGL(k_fine_stream<2>, g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
  return hipGetLastError();
}

hipError_t launch_em_union(const EMArgs& A, const int2* tiles, int ntiles, int ty, int nt,
                           hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 g(ntiles);
#define DMR_UNION_TILE(TY_)                                                                   \
  if (nt >= 1024) hipLaunchKernelGGL((k_fine_union<TY_, 1024>), g, dim3(1024), 0, st, A, tiles); \
  else hipLaunchKernelGGL((k_fine_union<TY_, 256>), g, dim3(256), 0, st, A, tiles)
  switch (ty) {
  case 4: DMR_UNION_TILE(4); break;
  case 8: DMR_UNION_TILE(8); break;
  default: DMR_UNION_TILE(16); break;
  }
#undef DMR_UNION_TILE
  return hipGetLastError();
}

hipError_t launch_cont_union(const ContArgs& A, const int2* tiles, int ntiles, int ty,
                             hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  switch (ty) {
  case 4: hipLaunchKernelGGL(k_cont_union<4>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  case 8: hipLaunchKernelGGL(k_cont_union<8>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  default: hipLaunchKernelGGL(k_cont_union<16>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  }
  return hipGetLastError();
}

hipError_t launch_em_union_batch(const EMArgs* args, const int2* blk, int nblk, int ty,
                                 hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  switch (ty) {
  case 4: hipLaunchKernelGGL(k_fine_union_batch<4>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  case 8: hipLaunchKernelGGL(k_fine_union_batch<8>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  default: hipLaunchKernelGGL(k_fine_union_batch<16>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  }
  return hipGetLastError();
}

hipError_t launch_cont_union_batch(const ContArgs* args, const int2* blk, int nblk, int ty,
                                   int slot, int update, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  switch (ty) {
  case 4: hipLaunchKernelGGL(k_cont_union_batch<4>, dim3(nblk), dim3(kThreads), 0, st, args, blk, slot, update); break;
  case 8: hipLaunchKernelGGL(k_cont_union_batch<8>, dim3(nblk), dim3(kThreads), 0, st, args, blk, slot, update); break;
  default: hipLaunchKernelGGL(k_cont_union_batch<16>, dim3(nblk), dim3(kThreads), 0, st, args, blk, slot, update); break;
  }
  return hipGetLastError();
}

hipError_t launch_prolong_union(const ProlongArgs& A, const int2* tiles, int ntiles, int ty,
                                hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  switch (ty) {
  case 4: hipLaunchKernelGGL(k_prolong_union<4>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  case 8: hipLaunchKernelGGL(k_prolong_union<8>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  default: hipLaunchKernelGGL(k_prolong_union<16>, dim3(ntiles), dim3(kThreads), 0, st, A, tiles); break;
  }
  return hipGetLastError();
}

// Width of the 4-row patch tiles: a tile's latency is set by its substep-1
// region (the tile plus a 7-cell halo), so small patches take the narrowest
// width whose tiles, with `others` blocks beside them, still fit one block
// per compute unit.  The width does not change any result.
int patch_tile_width(const EMArgs& F, int others) {
  const int nby = (F.T - F.B + 1 + 3) / 4;
  for (int tw = 16; tw < kTX; tw *= 2)
    if ((long)((F.R - F.L + 1 + tw - 1) / tw) * nby + others <= 256) return tw;
  return kTX;
}

// two substeps in the frame tile after the base step's launch (4-row tiles
// of width tw; r = 2: both substeps, r = 4: the second pair)
hipError_t launch_fine2_fast(const EMArgs& A, int tw, hipStream_t st) {
  if ((A.rf != 2 && A.rf != 4) || A.chz0 == nullptr || A.stix || A.st0x) return hipErrorInvalidValue;
  if (tw <= 0) tw = patch_tile_width(A, 0);
  const dim3 g((A.R - A.L + 1 + tw - 1) / tw, (A.T - A.B + 1 + 3) / 4), b(step_threads(false, 4));
  if (A.rf == 4) {
    if (tw == 16) hipLaunchKernelGGL((k_fine2_fast<16, true>), g, b, 0, st, A);
    else if (tw == 32) hipLaunchKernelGGL((k_fine2_fast<32, true>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_fine2_fast<kTX, true>), g, b, 0, st, A);
  } else {
    if (tw == 16) hipLaunchKernelGGL((k_fine2_fast<16, false>), g, b, 0, st, A);
    else if (tw == 32) hipLaunchKernelGGL((k_fine2_fast<32, false>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_fine2_fast<kTX, false>), g, b, 0, st, A);
  }
  return hipGetLastError();
}

hipError_t launch_fine2(const EMArgs& A, int ty, int nt, hipStream_t st) {
  if (A.rf == 4) {  // a pair of the four substeps, 1024 threads
    if (ty == 4) {
      const int tw = patch_tile_width(A, 0);
      const dim3 g((A.R - A.L + 1 + tw - 1) / tw, (A.T - A.B + 1 + 3) / 4);
      if (tw == 16) hipLaunchKernelGGL((k_fine2<4, 1024, false, true, 16>), g, dim3(1024), 0, st, A);
      else if (tw == 32) hipLaunchKernelGGL((k_fine2<4, 1024, false, true, 32>), g, dim3(1024), 0, st, A);
      else hipLaunchKernelGGL((k_fine2<4, 1024, false, true>), g, dim3(1024), 0, st, A);
      return hipGetLastError();
    }
    const dim3 g((A.R - A.L + 1 + kTX - 1) / kTX, (A.T - A.B + 1 + ty - 1) / ty);
    switch (ty) {
    case 8: hipLaunchKernelGGL((k_fine2<8, 1024, false, true>), g, dim3(1024), 0, st, A); break;
    default: hipLaunchKernelGGL((k_fine2<16, 1024, false, true>), g, dim3(1024), 0, st, A); break;
    }
    return hipGetLastError();
  }
  if (A.stn) {
    switch (ty) {
    case 4: DMR_LAUNCH_TILE_ST(k_fine2, 4, A, st); break;
    case 8: DMR_LAUNCH_TILE_ST(k_fine2, 8, A, st); break;
    default: DMR_LAUNCH_TILE_ST(k_fine2, 16, A, st); break;
    }
    return hipGetLastError();
  }
  if (ty == 4 && nt >= 1024) {
    const int tw = patch_tile_width(A, 0);
    const dim3 g((A.R - A.L + 1 + tw - 1) / tw, (A.T - A.B + 1 + 3) / 4);
    if (tw == 16) hipLaunchKernelGGL((k_fine2<4, 1024, false, false, 16>), g, dim3(1024), 0, st, A);
    else if (tw == 32) hipLaunchKernelGGL((k_fine2<4, 1024, false, false, 32>), g, dim3(1024), 0, st, A);
    else hipLaunchKernelGGL((k_fine2<4, 1024>), g, dim3(1024), 0, st, A);
    return hipGetLastError();
  }
  switch (ty) {
  case 4: DMR_LAUNCH_TILE(k_fine2, 4, nt, A, st); break;
  case 8: DMR_LAUNCH_TILE(k_fine2, 8, nt, A, st); break;
  default: DMR_LAUNCH_TILE(k_fine2, 16, nt, A, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_dmr_step(const EMArgs& C, const EMArgs& F, int seg, int depth, int ty,
                           int tw, hipStream_t st, bool r4) {
  if (r4 && (ty != 4 || C.stix)) return hipErrorInvalidValue;  // 4-row tiles, no replay
  const int waves_x = (C.R + 1 + 61) / 62;
  const int nseg = stream_segments(C.T, seg);
  const int nt = step_threads(C.stix != nullptr, ty);
  const int wpb = nt / 64;
  const int ncb = (waves_x * nseg + wpb - 1) / wpb;
  if (ty != 4) tw = kTX;  // narrow tiles: 4-row tiles only
  else if (tw <= 0) tw = patch_tile_width(F, ncb);
  const int nbx_f = (F.R - F.L + 1 + tw - 1) / tw;
  const int nby_f = (F.T - F.B + 1 + ty - 1) / ty;
  const dim3 g(ncb + nbx_f * nby_f), blk(nt);
#define DMR_STEP(D, T_, W_) hipLaunchKernelGGL((k_dmr_step<D, T_, false, W_>), g, blk, 0, st, C, F, seg, nseg, waves_x, ncb, nbx_f)
#define DMR_STEP_ST(D, T_, W_) hipLaunchKernelGGL((k_dmr_step<D, T_, true, W_>), g, blk, 0, st, C, F, seg, nseg, waves_x, ncb, nbx_f)
#define DMR_STEP_R4(D, W_) hipLaunchKernelGGL((k_dmr_step<D, 4, false, W_, true>), g, blk, 0, st, C, F, seg, nseg, waves_x, ncb, nbx_f)
  if (r4) {
    if (depth >= 4) { if (tw == 16) DMR_STEP_R4(4, 16); else if (tw == 32) DMR_STEP_R4(4, 32); else DMR_STEP_R4(4, kTX); }
    else { if (tw == 16) DMR_STEP_R4(2, 16); else if (tw == 32) DMR_STEP_R4(2, 32); else DMR_STEP_R4(2, kTX); }
  } else if (C.stix) {  // replay: stores for the adjoint
    if (depth >= 4) {
      if (ty == 4) { if (tw == 16) DMR_STEP_ST(4, 4, 16); else if (tw == 32) DMR_STEP_ST(4, 4, 32); else DMR_STEP_ST(4, 4, kTX); }
      else if (ty == 8) DMR_STEP_ST(4, 8, kTX); else DMR_STEP_ST(4, 16, kTX);
    } else {
      if (ty == 4) { if (tw == 16) DMR_STEP_ST(2, 4, 16); else if (tw == 32) DMR_STEP_ST(2, 4, 32); else DMR_STEP_ST(2, 4, kTX); }
      else if (ty == 8) DMR_STEP_ST(2, 8, kTX); else DMR_STEP_ST(2, 16, kTX);
    }
  } else if (depth >= 4) {
    if (ty == 4) { if (tw == 16) DMR_STEP(4, 4, 16); else if (tw == 32) DMR_STEP(4, 4, 32); else DMR_STEP(4, 4, kTX); }
    else if (ty == 8) DMR_STEP(4, 8, kTX); else DMR_STEP(4, 16, kTX);
  } else {
    if (ty == 4) { if (tw == 16) DMR_STEP(2, 4, 16); else if (tw == 32) DMR_STEP(2, 4, 32); else DMR_STEP(2, 4, kTX); }
    else if (ty == 8) DMR_STEP(2, 8, kTX); else DMR_STEP(2, 16, kTX);
  }
#undef DMR_STEP
#undef DMR_STEP_ST
#undef DMR_STEP_R4
  return hipGetLastError();
}

hipError_t launch_fine2_batch(const EMArgs* args, const int2* blk, int nblk, int ty, bool r4,
                              hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  const dim3 g(nblk), b(kFineThreads);
  if (r4) {
    if (ty == 4) hipLaunchKernelGGL((k_fine2_batch<4, true>), g, b, 0, st, args, blk);
    else if (ty == 8) hipLaunchKernelGGL((k_fine2_batch<8, true>), g, b, 0, st, args, blk);
    else hipLaunchKernelGGL((k_fine2_batch<16, true>), g, b, 0, st, args, blk);
  } else {
    if (ty == 4) hipLaunchKernelGGL((k_fine2_batch<4, false>), g, b, 0, st, args, blk);
    else if (ty == 8) hipLaunchKernelGGL((k_fine2_batch<8, false>), g, b, 0, st, args, blk);
    else hipLaunchKernelGGL((k_fine2_batch<16, false>), g, b, 0, st, args, blk);
  }
  return hipGetLastError();
}

hipError_t launch_dmr_step_batch(const EMArgs* cargs, const EMArgs* fargs, const int2* blk,
                                 int nblk, const float2* src, int k, int depth, int ty,
                                 hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  const dim3 g(nblk), b(kFineThreads);
#define DMR_SB(D, T_) hipLaunchKernelGGL((k_dmr_step_batch<D, T_>), g, b, 0, st, cargs, fargs, blk, src, k)
  if (depth >= 4) {
    if (ty == 4) DMR_SB(4, 4); else if (ty == 8) DMR_SB(4, 8); else DMR_SB(4, 16);
  } else {
    if (ty == 4) DMR_SB(2, 4); else if (ty == 8) DMR_SB(2, 8); else DMR_SB(2, 16);
  }
#undef DMR_SB
  return hipGetLastError();
}

hipError_t launch_em_stream_batch(const EMArgs* args, const int2* blk, int nblk,
                                  const float2* src, int k, int depth, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  if (depth >= 4)
    hipLaunchKernelGGL(k_em_stream_batch<4>, dim3(nblk), dim3(kThreads), 0, st, args, blk, src, k);
  else
    hipLaunchKernelGGL(k_em_stream_batch<2>, dim3(nblk), dim3(kThreads), 0, st, args, blk, src, k);
  return hipGetLastError();
}

hipError_t launch_em_batch(const EMArgs* args, const int2* blk, int nblk, int ty,
                           hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  switch (ty) {
  case 4: hipLaunchKernelGGL(k_fine_batch<4>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  case 8: hipLaunchKernelGGL(k_fine_batch<8>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  default: hipLaunchKernelGGL(k_fine_batch<16>, dim3(nblk), dim3(kFineThreads), 0, st, args, blk); break;
  }
  return hipGetLastError();
}

hipError_t launch_cont_batch(const ContArgs* args, const int2* blk, int nblk, bool fine,
                             int slot, int update, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  if (fine) hipLaunchKernelGGL(k_cont_batch<true>, dim3(nblk), dim3(kThreads), 0, st, args, blk, slot, update);
  else hipLaunchKernelGGL(k_cont_batch<false>, dim3(nblk), dim3(kThreads), 0, st, args, blk, slot, update);
  return hipGetLastError();
}

int stream_segments(int NY, int seg) {
  int nseg = (NY + 1 + seg - 1) / seg;
  if (nseg > 1 && (NY + 1) - (nseg - 1) * seg < 2) nseg--;  // no 1-row tail
  return nseg;
}

hipError_t launch_em_stream(const EMArgs& A, int seg, int depth, hipStream_t st) {
  const int waves = (A.R + 1 + 61) / 62;
  const int nseg = stream_segments(A.T, seg);
  const int nbx = (waves + kThreads / 64 - 1) / (kThreads / 64);
  dim3 g(nbx * nseg);
  if (A.stix) {  // replay: stores for the adjoint
    if (depth >= 4) hipLaunchKernelGGL((k_em_stream<4, true>), g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
    else hipLaunchKernelGGL((k_em_stream<2, true>), g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
  } else if (depth >= 4) {
    hipLaunchKernelGGL(k_em_stream<4>, g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
  } else {
    hipLaunchKernelGGL(k_em_stream<2>, g, dim3(kThreads), 0, st, A, seg, nseg, nbx);
  }
  return hipGetLastError();
}

// Sec. III.D threshold lines: one block walks the perimeter nodes of the
// patch; each side's flag is the OR over its line.
__global__ __launch_bounds__(1024) void k_line_flags(const float* __restrict__ n, int pitch,
                                                     int I0, int J0, int I1, int J1, float thr,
                                                     int* flags) {
  const int h = J1 - J0 + 1, w = I1 - I0 + 1;
  int fl = 0, fr = 0, fb = 0, ft = 0;
  for (int k = threadIdx.x; k < 2 * h + 2 * w; k += blockDim.x) {
    int i, j;
    if (k < h) { i = I0; j = J0 + k; }
    else if (k < 2 * h) { i = I1; j = J0 + k - h; }
    else if (k < 2 * h + w) { i = I0 + k - 2 * h; j = J0; }
    else { i = I0 + k - 2 * h - w; j = J1; }
    const bool hit = n[(size_t)j * pitch + i] > thr;
    if (k < h) fl |= hit;
    else if (k < 2 * h) fr |= hit;
    else if (k < 2 * h + w) fb |= hit;
    else ft |= hit;
  }
  fl = __syncthreads_or(fl);
  fr = __syncthreads_or(fr);
  fb = __syncthreads_or(fb);
  ft = __syncthreads_or(ft);
  if (threadIdx.x < 4) {
    const int v = threadIdx.x == 0 ? fl : threadIdx.x == 1 ? fr : threadIdx.x == 2 ? fb : ft;
    flags[threadIdx.x] = v ? 1 : 0;
  }
}

hipError_t launch_line_flags(const float* n, int pitch, int I0, int J0, int I1, int J1,
                             float thr, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_line_flags, dim3(1), dim3(1024), 0, st, n, pitch, I0, J0, I1, J1, thr,
                     flags);
  return hipGetLastError();
}

hipError_t launch_cont(const ContArgs& A, bool fine, hipStream_t st) {
  const int nx = A.R - A.L + 1, ny = A.T - A.B + 1;
  dim3 g((nx + kTX - 1) / kTX, (ny + kThreads / kTX - 1) / (kThreads / kTX));
  if (fine) hipLaunchKernelGGL(k_cont<true>, g, dim3(kThreads), 0, st, A);
  else hipLaunchKernelGGL(k_cont<false>, g, dim3(kThreads), 0, st, A);
  return hipGetLastError();
}

// both levels' continuity in one launch (r = 2 rectangle; C.pL..C.pT set)
hipError_t launch_cont2(const ContArgs& C, const ContArgs& F, hipStream_t st) {
  if ((F.rf != 2 && F.rf != 4) || F.act || C.pR <= C.pL || C.pT <= C.pB) return hipErrorInvalidValue;
  // the boundary block: one coarse node and r patch nodes per thread
  const long nfn = 2L * (F.R - F.L + 1) + 2L * (F.T - F.B - 1);
  const long ncn = 2L * (C.pR - C.pL + 1) + 2L * (C.pT - C.pB - 1);
  if (nfn > (long)F.rf * kCont2Threads || ncn > kCont2Threads) return hipErrorInvalidValue;
  const int rows = kCont2Threads / kTX;
  const int gxc = (C.R - C.L + 1 + kTX - 1) / kTX, gyc = (C.T - C.B + 1 + rows - 1) / rows;
  const int gxf = (F.R - F.L + 1 + kTX - 1) / kTX, gyf = (F.T - F.B + 1 + rows - 1) / rows;
  const dim3 g(gxc * gyc + gxf * gyf + 1);
  if (F.rf == 4)
    hipLaunchKernelGGL(k_cont2<4>, g, dim3(kCont2Threads), 0, st, C, F, gxc, gxc * gyc, gxf, gxf * gyf);
  else
    hipLaunchKernelGGL(k_cont2<2>, g, dim3(kCont2Threads), 0, st, C, F, gxc, gxc * gyc, gxf, gxf * gyf);
  return hipGetLastError();
}

hipError_t launch_regrid_test(const FlagArgs& F, const ScanArgs& S, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_blocks, dim3(F.NBx, F.NBy), dim3(256), 0, st, F);
  hipLaunchKernelGGL(k_scan_bbox, dim3(1), dim3(1024), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_prolong(const ProlongArgs& A, hipStream_t st) {
  const int nx = A.R - A.L + 1, ny = A.T - A.B + 1;
  dim3 g((nx + kTX - 1) / kTX, (ny + kThreads / kTX - 1) / (kThreads / kTX));
  hipLaunchKernelGGL(k_prolong, g, dim3(kThreads), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_gather(const float* src, int pitch, int i0, int j0, int cols,
                         int rows, float scale, float* dst, hipStream_t st) {
  dim3 g((cols + 255) / 256, rows);
  hipLaunchKernelGGL(k_gather, g, dim3(256), 0, st, src, pitch, i0, j0, cols,
                     rows, scale, dst);
  return hipGetLastError();
}

hipError_t launch_scatter(const float* src, int cols, int rows, float scale,
                          float* dst, int pitch, int i0, int j0, hipStream_t st) {
  dim3 g((cols + 255) / 256, rows);
  hipLaunchKernelGGL(k_scatter, g, dim3(256), 0, st, src, cols, rows, scale,
                     dst, pitch, i0, j0);
  return hipGetLastError();
}

hipError_t launch_ring_sum(const float* ring, size_t plane, int pitch, int i0,
                           int j0, int cols, int rows, float* dst,
                           hipStream_t st) {
  dim3 g((cols + 255) / 256, rows);
  hipLaunchKernelGGL(k_ring_sum, g, dim3(256), 0, st, ring, plane, pitch, i0,
                     j0, cols, rows, dst);
  return hipGetLastError();
}

}  // namespace dmr
