// dmr_kernels.h -- argument blocks and launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dmr {

constexpr int kTX = 64;        // tile width in nodes: one wavefront per row
constexpr int kThreads = 256;  // threads per tile
constexpr int kRing = 8;       // window blocks per period
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
  float inv_namb, De, Da;
  int d_const_mode;
  float d_const;
  int* err;        // 64 flags, set on non-finite values
  float* cn1;      // fine level: coarse density after its update
  int cpitch;
  int nbx;         // batched launches: blocks per row of blocks
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
  const float *chz, *chz_prev, *cex, *cey, *cjx, *cjy, *cn, *cacc, *cring;
  float *hz, *ex, *ey, *jx, *jy, *n, *acc, *ring;
};

hipError_t launch_em(const EMArgs& A, bool fine, int ty, hipStream_t st);
// base level, column-streaming kernel; seg = rows per segment (>= 2)
hipError_t launch_em_stream(const EMArgs& A, int seg, int depth, hipStream_t st);
int stream_segments(int NY, int seg);
// batched forms: blk[b] = (instance, block index within the instance)
hipError_t launch_em_stream_batch(const EMArgs* args, const int2* blk, int nblk,
                                  const float2* src, int k, int depth, hipStream_t st);
hipError_t launch_em_batch(const EMArgs* args, const int2* blk, int nblk, int ty,
                           hipStream_t st);
hipError_t launch_cont_batch(const ContArgs* args, const int2* blk, int nblk, bool fine,
                             int slot, int update, hipStream_t st);
hipError_t launch_cont(const ContArgs& A, bool fine, hipStream_t st);
hipError_t launch_regrid_test(const FlagArgs& F, const ScanArgs& S, hipStream_t st);
hipError_t launch_prolong(const ProlongArgs& A, hipStream_t st);
hipError_t launch_gather(const float* src, int pitch, int i0, int j0, int cols,
                         int rows, float scale, float* dst, hipStream_t st);
hipError_t launch_scatter(const float* src, int cols, int rows, float scale,
                          float* dst, int pitch, int i0, int j0, hipStream_t st);
hipError_t launch_ring_sum(const float* ring, size_t plane, int pitch, int i0,
                           int j0, int cols, int rows, float* dst,
                           hipStream_t st);

}  // namespace dmr
