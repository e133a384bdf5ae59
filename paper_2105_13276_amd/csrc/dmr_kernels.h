// dmr_kernels.h -- argument blocks and launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dmr {

constexpr int kTX = 64;        // tile width in nodes: one wavefront per row
constexpr int kThreads = 256;  // threads per tile
constexpr int kFineThreads = 1024;  // threads per patch tile (phases run from LDS)
constexpr int kTileSgprs = 72;  // scalar-register cap of the 1024-thread tile kernels
// continuity-adjoint tiles: node columns x rows per block, threads per block
// (the tape sizes its per-block partial sums from the tile)
constexpr int kAdjContTX = 32, kAdjContTY = 5, kAdjContThreads = 256;
// threads per block of the combined step: 512 for its 4-row patch tiles (one
// frame position per thread on small patches, and half as many base-level
// waves per compute unit), else the patch tile's 1024
constexpr int step_threads(bool store, int ty) { return (!store && ty == 4) ? 512 : kFineThreads; }
constexpr int kRing = 8;       // window blocks per period
// union-of-blocks level: Eq. (5b) values one tile hands from substep 1 to the
// last substep (4 block columns x (16+1) rows + 2 block rows x (kTX+1))
constexpr int kCfbStride = 4 * 17 + 2 * (kTX + 1);
constexpr int kBcMur = 0;
constexpr int kSrcSteps = 256;  // incident-value table length of the batched form

struct EMArgs {
  const float *hz0, *ex0, *ey0, *jx0, *jy0;  // state at step n (read)
  float *hz1, *ex1, *ey1, *jx1, *jy1;        // state at step n+1 (written)
  const float* n;                            // density at the nodes
  float* acc;                                // window accumulator (in place)
  int pitch;
  int L, B, R, T;  // active cells [L,R) x [B,T); nodes [L,R] x [B,T]
  float S;         // c dt / dx
  float c1;        // (1 + a) / 2
  float a;         // exp(-nu_m dt)
  float kn;        // dt b / (4 eps0), times n_e gives k
  float cmur;      // (S - 1) / (S + 1)
  // base level
  int bc_x, bc_y;
  int is;                // TF/SF node column (<= 0: none)
  float ey_src, hz_src;  // incident Ey(x_s, t^n), eta0 Hz(x_s - dx/2, t^{n+1/2})
  // fine level: coarse E before / after the coarse step, time fraction
  const float *cex0, *cey0, *cex1, *cey1;
  int cpitch;
  float frac;
  float gamma;  // fine-patch E hyper-diffusion coefficient (<= 0: off)
  // fine level, last substep: coarse targets of the fine -> coarse transfer
  int restrict_on;
  float *chz, *cex, *cey, *cjx, *cjy;
  // batched launches: tiles per row of tiles, and the streaming segments
  int nbx, seg, nseg;
  // base level in the combined step: coarse entities [sL,sR) x [sB,sT)
  // strictly inside the patch are not stored (the patch tiles write them)
  int skip_on, sL, sB, sR, sT;
  // patch tiles of the combined step: coarse state entering the step, for
  // the coarse E after it on the patch boundary lines (computed locally)
  const float *chz0, *cjx0, *cjy0, *cn0;
  float cS, cc1, ckn, cey_src, chz_src;
  int cis, cnx, cny;
  // refinement factor of the patch (0 or 2: r = 2; 4).  r = 4: substep r/2
  // saves its new Hz (hz_save), the last substep reads it back (hz_lo): the
  // two half levels around coarse n+1/2 are after substeps r/2 and r/2 + 1
  int rf;
  float* hz_save;
  const float* hz_lo;
  // replay for the adjoint (null: off): the step's values it needs, written
  // at the entity's own position.  Base level: E entering (sti), E after the
  // step before the fine -> coarse transfer (sto), n.  Patch (both
  // substeps): E entering substep 1 (st0), after substep 1 (st1), after
  // substep 2 (st2, nullable), n.
  float *stix, *stiy, *stox, *stoy, *stn;
  float *st0x, *st0y, *st1x, *st1y, *st2x, *st2y;
  // fine level as a union of blocks (act non-null): active blocks
  // [nbky][nbkx] of 2^fbs x 2^fbs fine cells; L = B = 0, R x T the fine
  // domain; the tiles come from a list
  const uint8_t* act;
  int fbs, nbkx, nbky;
  // union, r = 2: substep 1 writes the Eq. (5b) values of the last substep
  // (frac = 1) per listed tile (cfb_next), which reads them back (cfb_prev)
  // instead of the coarse E its own fine -> coarse transfer rewrites
  float* cfb_next;
  const float* cfb_prev;
  const int2* utiles;  // batched union levels: the instance's tile list
};

struct ContArgs {
  const float* n0;
  float* n1;
  float* acc;
  float* ring;
  size_t plane;
  int pitch;
  int L, B, R, T;  // node region
  int slot, update;
  float inv_spp;   // 1 / steps per period
  float dtn;       // continuity step
  float inv_dx2;
  float eeff_p2;   // (1/(1 + w^2/nu^2)) / (100 p)^2
  float half_beta, att, nuA;
  // Townsend source (town): nu = tK y exp(-tB / y) - tatt, y = E_eff/(100 p);
  // recombination r_ei (0: none)
  int town;
  float tK, tB, tatt, rei;
  float inv_namb, De, Da;
  int d_const_mode;
  float d_const;
  int* err;        // 64 flags, set on non-finite values
  float* cn1;      // fine level: coarse density after its update
  int cpitch;
  int rf;          // fine level: refinement factor (0 or 2: r = 2; 4)
  int nbx;         // batched launches: blocks per row of blocks
  // fine level as a union of blocks (as in EMArgs)
  const uint8_t* act;
  int fbs, nbkx, nbky;
  const int2* utiles;  // batched union levels: the instance's tile list
  // one-launch continuity of both levels (k_cont2): the patch's node extent
  // in coarse nodes (pL < pR), whose boundary-line nodes a block of their own
  // updates; 0 / 0: off
  int pL, pB, pR, pT;
};

struct FlagArgs {
  const float* n;
  int pitch, NX, NY, Bk, NBx, NBy;
  float thr, flo, g2;
  uint8_t* bflag;
};

struct ScanArgs {
  const uint8_t* bflag;
  int NB, NBx, NBy;
  int32_t *scan, *list;
  int* desc;
};

struct ProlongArgs {
  int L, B, R, T;      // new patch, fine cells
  int oL, oB, oR, oT;  // old patch (oR <= oL: none)
  int pitch, cpitch;
  size_t plane, cplane;
  int keep_n;
  int rf;              // refinement factor (0 or 2: r = 2; 4)
  const float *chz, *chz_prev, *cex, *cey, *cjx, *cjy, *cn, *cacc, *cring;
  float *hz, *ex, *ey, *jx, *jy, *n, *acc, *ring;
  // fine level as a union of blocks: active blocks after (act) and before
  // (act_old) the growth, as in EMArgs
  const uint8_t *act, *act_old;
  int fbs, nbkx, nbky;
  const float* seed;  // union with keep_n: the fine density of new nodes (pitched)
};

// patch substep kernel, 64 x ty tiles of nt threads (256 or 1024)
hipError_t launch_em(const EMArgs& A, bool fine, int ty, int nt, hipStream_t st);
// the same substep on the union of blocks: the 64 x ty tiles (tile column,
// tile row) listed in tiles[ntiles]
hipError_t launch_em_union(const EMArgs& A, const int2* tiles, int ntiles, int ty, int nt,
                           hipStream_t st);
// continuity on the fine union of blocks over the same tile list (64 x ty)
hipError_t launch_cont_union(const ContArgs& A, const int2* tiles, int ntiles, int ty,
                             hipStream_t st);
// batched union levels (every instance a union): blk[b] = (instance, index in
// the instance's tile list utiles), 64 x ty tiles for every instance
hipError_t launch_em_union_batch(const EMArgs* args, const int2* blk, int nblk, int ty,
                                 hipStream_t st);
hipError_t launch_cont_union_batch(const ContArgs* args, const int2* blk, int nblk, int ty,
                                   int slot, int update, hipStream_t st);
// prolongation into the blocks new to the union, over the listed 64 x ty tiles
hipError_t launch_prolong_union(const ProlongArgs& A, const int2* tiles, int ntiles, int ty,
                                hipStream_t st);
// both patch substeps of a coarse step in one launch: reads buffer 0 (hz0..),
// writes buffer 1 (hz1..), A.frac = time fraction of substep 1, restriction on
hipError_t launch_fine2(const EMArgs& A, int ty, int nt, hipStream_t st);
hipError_t launch_fine2_fast(const EMArgs& A, int tw, hipStream_t st);
// base-level step (C, with the patch's coarse entities skipped) and both patch
// substeps (F, coarse boundary E computed in the tiles) in one launch
hipError_t launch_dmr_step(const EMArgs& C, const EMArgs& F, int seg, int depth, int ty,
                           int tw, hipStream_t st, bool r4 = false);
// base level, column-streaming kernel; seg = rows per segment (>= 2)
hipError_t launch_em_stream(const EMArgs& A, int seg, int depth, hipStream_t st);
// one patch substep (rectangle, r = 2) in column-streaming form, for large
// patches; seg = rows per segment (even), depth = rows of loads in flight
hipError_t launch_fine_stream(const EMArgs& A, int seg, int depth, hipStream_t st);
// threshold lines of the patch sides (left I0, right I1, bottom J0, top J1):
// flags[q] = 1 if a base node on line q has n > thr (one block, 4 ints)
hipError_t launch_line_flags(const float* n, int pitch, int I0, int J0, int I1, int J1,
                             float thr, int* flags, hipStream_t st);
int stream_segments(int NY, int seg);
// batched forms: blk[b] = (instance, block index within the instance)
hipError_t launch_em_stream_batch(const EMArgs* args, const int2* blk, int nblk,
                                  const float2* src, int k, int depth, hipStream_t st);
hipError_t launch_em_batch(const EMArgs* args, const int2* blk, int nblk, int ty,
                           hipStream_t st);
// batched two-substep patch launch over the same (instance, tile) table as
// launch_em_batch (r4: a pair of the four r = 4 substeps)
hipError_t launch_fine2_batch(const EMArgs* args, const int2* blk, int nblk, int ty, bool r4,
                              hipStream_t st);
// batched combined step: blk[b] = (instance, g >= 0: group of 16 base waves,
// g < 0: patch tile -1 - g); cargs the base levels (patch entities skipped),
// fargs the patch tiles (coarse boundary E computed locally)
hipError_t launch_dmr_step_batch(const EMArgs* cargs, const EMArgs* fargs, const int2* blk,
                                 int nblk, const float2* src, int k, int depth, int ty,
                                 hipStream_t st);
hipError_t launch_cont_batch(const ContArgs* args, const int2* blk, int nblk, bool fine,
                             int slot, int update, hipStream_t st);
hipError_t launch_cont(const ContArgs& A, bool fine, hipStream_t st);
hipError_t launch_cont2(const ContArgs& C, const ContArgs& F, hipStream_t st);
hipError_t launch_regrid_test(const FlagArgs& F, const ScanArgs& S, hipStream_t st);
hipError_t launch_prolong(const ProlongArgs& A, hipStream_t st);
hipError_t launch_gather(const float* src, int pitch, int i0, int j0, int cols,
                         int rows, float scale, float* dst, hipStream_t st);
hipError_t launch_scatter(const float* src, int cols, int rows, float scale,
                          float* dst, int pitch, int i0, int j0, hipStream_t st);
hipError_t launch_ring_sum(const float* ring, size_t plane, int pitch, int i0,
                           int j0, int cols, int rows, float* dst,
                           hipStream_t st);

// ---------------------------------------------------------------------------
// Adjoint (reverse-mode) kernels.  Adjoint planes share the layout of the
// level they belong to.  "lam" = dF/d(value) for the objective F.
// ---------------------------------------------------------------------------
struct AdjEMArgs {
  int L, B, R, T, pitch;
  float S, c1, a, kn, cmur, gamma;
  int fine, bc_x, bc_y, is;
  const float *exi, *eyi;  // E entering the (sub)step (fine: before the filter)
  const float *exo, *eyo;  // E leaving it (base: before the fine -> coarse transfer)
  const float* n;
  const float* lhz_in;     // lam of Hz leaving the step
  float* lhz_out;          // lam of Hz entering it
  const float *lex, *ley, *ljx, *ljy;  // lam of E, J leaving the step
  float *lex_o, *ley_o, *ljx_o, *ljy_o;  // lam of E, J entering it (other buffers)
  const float* lacc;
  float* hz_extra;         // base: added to lam Hz entering, then cleared (nullable)
  float *gx, *gy;          // patch, out: g per edge (G on boundary edges)
  float* ln;               // lam n (accumulated)
  float *src_e, *src_h;    // base: per-row source sensitivities (nullable)
  // patch, last substep: the fine -> coarse transfer transposed, folded into
  // the loads (the coarse lam of the entities strictly inside the coarse
  // patch I0..I1 x J0..J1 goes to the fine entities averaged into them)
  int I0, J0, I1, J1, cpitch;
  const float *rhz, *rex, *rey, *rjx, *rjy;  // coarse lam (null: no transfer)
  // base level with a patch (has_patch): the lam inputs of the entities
  // strictly inside it read as zero (their lam went to the patch), and the
  // Eq. (5b) boundary values transposed are gathered from the patch g of
  // the two substeps on the fine cells fL..fR x fB..fT
  int has_patch, fL, fB, fR, fT, fpitch;
  const float *g2x, *g2y;  // patch g of substep 2 (its boundary G)
  // substep 1's boundary G is computed here from its inputs (it does not
  // depend on substep 1's H'), so substep 1 can run in the same launch:
  // lam E, lam J leaving substep 1, E after it, lam acc, n, and the patch kn
  const float *s1ex, *s1ey, *s1jx, *s1jy, *s1exo, *s1eyo, *s1acc, *s1n;
  float s1kn;
};

struct AdjGrowArgs {
  int L, B, R, T;      // new patch, fine cells
  int oL, oB, oR, oT;  // old patch (oR <= oL: none)
  int cL, cB, cR, cT;  // coarse node positions to gather into
  int cNX, cNY;        // coarse cells
  int pitch, cpitch;
  size_t plane, cplane;
  int with_n;
  const float *lhz, *lex, *ley, *ljx, *ljy, *ln, *lacc, *lring;   // fine lam
  float *chz, *chz_prev, *cex, *cey, *cjx, *cjy, *cn, *cacc, *cring;  // coarse lam
};

struct AdjContArgs {
  int L, B, R, T, pitch;
  size_t plane;
  int fine, slot, update;
  float inv_spp, dtn, inv_dx2, eeff_p2, half_beta, att, nuA, nu_m, ln_c;
  float inv_namb, De, Da;
  int d_const_mode;
  float d_const;
  // Townsend source (town) and recombination (rei), as in ContArgs
  int town;
  float tK, tB, tatt, rei;
  const float* n;   // density entering the continuity step
  const float* e2;  // E_rms^2 the step used
  float* ln;        // lam n leaving (entering: ln_o)
  float* ln_o;      // lam n entering the step (another buffer)
  float* lacc;
  float* lring;
  double* part;     // per-block (dF/dA, dF/dbeta) partial sums
};

struct AdjInjArgs {
  int I0, J0, I1, J1, pitch, cpitch;
  float *lcn, *lfn;
};

struct CopyJob {
  const float* src;
  float* dst;
  size_t n;  // floats, a multiple of 4
};
constexpr int kMaxCopyJobs = 40;
struct CopyJobs {
  CopyJob job[kMaxCopyJobs];
  int count;
};

hipError_t launch_adj_em(const AdjEMArgs& A, hipStream_t st);
// patch substep 1 (F) and the base level (C) of one base step in one launch
hipError_t launch_adj_em_pair(const AdjEMArgs& F, const AdjEMArgs& C, hipStream_t st);
hipError_t launch_adj_grow(const AdjGrowArgs& A, hipStream_t st);
hipError_t launch_adj_grow_clear(const AdjGrowArgs& A, float* lhz, float* lex, float* ley,
                                 float* ljx, float* ljy, float* ln, float* lacc,
                                 float* lring, hipStream_t st);
// rows x cols block between two pitched arrays
hipError_t launch_copy2d(const float* src, int spitch, int si0, int sj0, float* dst,
                         int dpitch, int di0, int dj0, int cols, int rows, hipStream_t st);
hipError_t launch_adj_inj(const AdjInjArgs& A, hipStream_t st);
// continuity adjoint; returns the number of partial pairs written
// continuity step transposed on the patch (F, if has_f) and the base level
// (C) in one launch; nparts: the partial-sum blocks written from A.part on
hipError_t launch_adj_cont(const AdjContArgs& F, const AdjContArgs& C, int has_f, int* nparts,
                           hipStream_t st);
hipError_t launch_adj_close(const AdjContArgs& A, hipStream_t st);
hipError_t launch_copy(const CopyJobs& J, hipStream_t st);
hipError_t launch_ring_e2(const float* ring, size_t plane, int pitch, int L, int B,
                          int R, int T, float* dst, hipStream_t st);
// out[0] += sum_k u[2k] sum_j src_e[k][j] + u[2k+1] sum_j src_h[k][j]
// (src_e of step k at src + k*step_pitch, src_h rows floats after it);
// out[1..2] += sum of the (dF/dA, dF/dbeta) partial pairs
hipError_t launch_adj_reduce(const float* src, int nsteps, int step_pitch, int rows,
                             const double* u, const double* part, int nparts, double* out,
                             hipStream_t st);
// sum over a pitched region of w (dense, cols x rows) times a (pitched)
hipError_t launch_wdot(const float* w, const float* a, int pitch, int i0, int j0,
                       int cols, int rows, double* part, double* out, hipStream_t st);

}  // namespace dmr
