/*
 * dmr.h -- C ABI of the MI355X (gfx950) library for the coupled EM / plasma
 * fluid update with dynamic mesh refinement of Ghosh & Chaudhury,
 * "Efficient Dynamic Mesh Refinement Technique for Simulation of HPM
 * Breakdown induced Plasma Pattern Formation".
 *
 * The library advances, on one GPU and one HIP stream:
 *   - the Yee TE_z update of Hz, Ex, Ey (Eqs. (1)-(2), Sec. II.B), with a
 *     total-field/scattered-field plane-wave source entering from the left
 *     and first-order Mur outer boundaries (Sec. II.B, Fig. 1 caption);
 *   - the electron current dJ/dt = -nu_m J + (e^2 n/m) E (Eq. (3) in current
 *     form, J = -e n v), coupled semi-implicitly to E;
 *   - the one-period E_rms window and the continuity step
 *     dn/dt = div(D_eff grad n) + nu(E_eff) n (Eq. (4), Sec. II.A), every 1/8
 *     of a wave period;
 *   - one fine patch over the plasma (Sec. III), r = 2 or 4: r fine substeps
 *     per coarse step, tangential E on the coarse/fine boundary by Eq. (5b),
 *     fine -> coarse transfer after the last substep, density transfers at
 *     each continuity step, and the self-aware growth test of Sec. III.A-D
 *     (threshold and gradient-length flags on square blocks, prefix-sum
 *     compaction, bounding-box growth, Eq. (5a) prolongation); or a fine
 *     level made of the flagged blocks themselves (DMR_RULE_UNION).
 *
 * Conventions for every call:
 *   - Return value: DMR_OK (0) or a negative DMR_E* code; the text of the
 *     last error of a handle is in dmr_last_error().  Nothing aborts or
 *     throws across the ABI.  A handle is not thread-safe.
 *   - The library allocates no device memory.  The caller passes one device
 *     workspace of at least dmr_workspace_bytes() bytes that must outlive the
 *     handle, and the HIP stream (hipStream_t as void*, NULL = default
 *     stream) on which all work is queued.
 *   - Calls that only queue work (dmr_step) return before it ends; calls
 *     that hand data to the host synchronise the stream.
 *   - Fields are float32, SI units, row-major with y rows and x fastest,
 *     no padding:
 *        DMR_HZ        [ny  ][nx  ]  cell centres (i+1/2, j+1/2)   A/m
 *        DMR_EX/JX     [ny+1][nx  ]  x-edges      (i+1/2, j)   V/m, A/m^2
 *        DMR_EY/JY     [ny  ][nx+1]  y-edges      (i, j+1/2)   V/m, A/m^2
 *        DMR_N, DMR_ACC, DMR_ERMS2 [ny+1][nx+1] nodes (i, j)  m^-3, V^2/m^2
 *        DMR_RING      8 planes of nodes (mean E^2 of each 1/8 period)
 *     Level 0 is the base (coarse, or the only) mesh; level 1 is the fine
 *     patch, whose nx, ny are its size in fine cells (dmr_field_dims).
 */
#ifndef DMR_H
#define DMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMR_OK 0
#define DMR_EINVAL (-1)    /* bad argument, or a stability/shape rule broken */
#define DMR_ENOMEM (-2)    /* workspace too small */
#define DMR_EHIP (-3)      /* a HIP call failed (also late async errors) */
#define DMR_EUNSTABLE (-4) /* non-finite density or window detected */

enum { DMR_BC_MUR = 0, DMR_BC_PEC = 1 };
enum { DMR_UNIFORM = 0, DMR_STATIC = 1, DMR_DYNAMIC = 2 };
enum { DMR_RULE_BLOCKS = 0, DMR_RULE_LINES = 1, DMR_RULE_UNION = 2 };
enum { DMR_SOURCE_POWER = 0, DMR_SOURCE_TOWNSEND = 1 };
enum { DMR_D_BLEND = 0, DMR_D_CONST = 1 };
enum {
  DMR_HZ = 0, DMR_EX = 1, DMR_EY = 2, DMR_JX = 3, DMR_JY = 4,
  DMR_N = 5, DMR_ACC = 6, DMR_ERMS2 = 7, DMR_RING = 8
};

/* The problem statement of Sec. II.B / Sec. IV: domain, incident wave, gas,
 * seed, resolution, refinement factor and refinement thresholds.  Plain old
 * data, copied at dmr_create; struct_size must be sizeof(dmr_params). */
typedef struct dmr_params {
  uint32_t struct_size;
  int32_t nx, ny;            /* base-level cells (domain = nx*dx by ny*dx) */
  int32_t cells_per_lambda;  /* base-level N_lambda (dx = lambda/N) */
  int32_t r;                 /* refinement factor, 2 or 4 (the combined one-launch
                                step, the union level and the adjoint: 2; a
                                batch: one r for all its refined instances) */
  int32_t block;             /* regrid block edge in base cells (divides nx, ny) */
  int32_t regrid_every;      /* base steps between growth tests */
  int32_t tfsf_i;            /* source node column (base cells), 1..nx-1 */
  int32_t ramp_periods;      /* sin^2 turn-on of the incident wave */
  int32_t bc_x, bc_y;        /* DMR_BC_MUR or DMR_BC_PEC */
  int32_t mode;              /* DMR_UNIFORM, DMR_STATIC, DMR_DYNAMIC */
  int32_t static_ext[4];     /* I0, J0, I1, J1 base cells (DMR_STATIC) */
  int32_t d_mode;            /* DMR_D_BLEND (default) or DMR_D_CONST */
  int32_t continuity_on;     /* 0: density and window frozen */
  int32_t pad_;
  double freq_hz;            /* incident frequency */
  double erms_over_ebd;      /* incident rms field / breakdown field */
  double p_torr;             /* gas pressure; nu_m = 5.3e9 p (Sec. II.A) */
  double A_ion, beta_ion;    /* nu = nu_m A [(E_eff/p)^beta - (E_cr/p)^beta] */
  double ecr_over_p;         /* E_cr/p, V/(cm Torr) */
  double te_ev, ti_ev;       /* electron / ion temperature, eV */
  double mu_i_760;           /* ion mobility at 760 Torr, m^2/(V s) */
  double L_amb;              /* ambipolar transition length, m */
  double d_const;            /* D for DMR_D_CONST, m^2/s */
  double n_thr_over_nc;      /* threshold density / critical density */
  double grad_thr;           /* flag where |grad n| dx / n > grad_thr */
  double n_floor_over_nc;    /* gradient test only above this density */
  double courant;            /* S = c dt/dx, same on both levels, <= 1/sqrt 2 */
  double fine_filter;        /* gamma of the weak 4th-order hyper-diffusion of
                                the patch's interior E, applied before each
                                fine substep (1e-3 suppresses the slow growth
                                of sub-coarse modes at the interface for the
                                patch shapes tried; 0: off; at most 1/64) */
  /* growth rule of DMR_DYNAMIC (Sec. III.D):
   *   DMR_RULE_BLOCKS  flag nodes (n_thr_over_nc, grad_thr, n_floor_over_nc),
   *                    OR over block x block cells, prefix-sum compaction,
   *                    bounding box of the old patch and the flagged blocks;
   *   DMR_RULE_LINES   the threshold lines: the initial patch is m_lx x m_ly
   *                    base cells centred on the seed's peak node; at each
   *                    test, a side of the patch whose boundary line carries a
   *                    node with n > n_line moves out by m_ex (left / right
   *                    sides) or m_ey (bottom / top);
   *   DMR_RULE_UNION   the flags of DMR_RULE_BLOCKS, but the fine level is
   *                    the union of the flagged blocks themselves instead of
   *                    their bounding box (several separate regions; Sec.
   *                    III.A/B flags, Sec. III.C transfers on every
   *                    coarse/fine boundary edge).  r = 2, block a power of
   *                    two >= 8; with DMR_STATIC the fine level starts as the
   *                    blocks of static_ext (whole blocks).  Not supported by
   *                    the adjoint; in a batch, every instance or none.
   * All keep the fine level one block clear of the outer boundary and right
   * of the source line by one block, and only grow it. */
  int32_t regrid_rule;
  int32_t m_lx, m_ly, m_ex, m_ey;  /* base cells (DMR_RULE_LINES) */
  int32_t pad2_;
  double n_line;             /* threshold density on the lines, m^-3 */
  /* source of Eq. (4): n (nu_i - nu_a) - r_ei n^2 with
   *   DMR_SOURCE_POWER     nu_i - nu_a = nu_m A [(E_eff/p)^beta - (E_cr/p)^beta]
   *   DMR_SOURCE_TOWNSEND  nu_i - nu_a = gamma v_d - nu_att, Townsend
   *                        gamma = A_town p exp(-B_town p / E_eff) (A_town in
   *                        1/(cm Torr), B_town in V/(cm Torr), E_eff/p in
   *                        V/(cm Torr)), drift v_d = e E_eff / (m nu_m),
   *                        attachment nu_att (1/s)
   * and recombination r_ei = beta_rec 1e-13 (300 K / T_e)^(1/2) m^3/s
   * (T_e = te_ev in kelvin; beta_rec in [0, 2], 0: none).  The adjoint
   * supports both sources, with or without recombination. */
  int32_t source_model;
  int32_t pad3_;
  double A_town, B_town, nu_att, beta_rec;
} dmr_params;

typedef struct dmr_sim dmr_sim;

/* Host only, no device call: the scalars the library derives from *p before
 * a run, as dmr_create computes them, in this order: omega = 2 pi f; lambda
 * = c/f; the base level's dx = lambda/cells_per_lambda and dt = S dx/c;
 * nu_m = 5.3e9 p (Sec. II.A); the critical density n_c = m_e eps0 omega^2 /
 * e^2; the effective-field factor 1/(1 + (omega/nu_m)^2) (Sec. II.A); the rms
 * breakdown field E_bd and the incident amplitude E0 = sqrt 2 (E_rms/E_bd)
 * E_bd; D_e and D_a and the ambipolar density scale of Eq. (4); the base
 * level's Drude decay a = exp(-nu_m dt) and drive b = e^2 (1 - a)/(m_e nu_m)
 * (Eq. (3), both as the kernels receive them in float32); the numerical
 * wavenumber of the incident wave (Sec. II.B); the ionisation model's
 * nu_m A (E_cr/p)^beta (float32 product, as the kernels use it); and the base
 * steps per period.  out receives the first min(n_out, 17) of these.
 * EINVAL on bad params or out == NULL. */
int dmr_derived(const dmr_params *p, double *out, int n_out);

/* Bytes of device workspace the problem needs, sized for a patch covering
 * the whole domain so that growth never reallocates.  EINVAL on bad params. */
int dmr_workspace_bytes(const dmr_params *p, size_t *bytes);

/* Create a simulation at t = 0: fields and current zero, density from the
 * seeds (the Gaussian of Sec. IV, or any field), and for DMR_DYNAMIC the
 * growth test run once to place the initial patch (Sec. III.D).
 *   seed_base  host float64 node densities of level 0, [ny+1][nx+1]; NULL = 0
 *   seed_fine  host float64 densities on the full-domain fine grid
 *              [r*ny+1][r*nx+1], used for the patch built at t = 0;
 *              NULL = interpolate from seed_base (Eq. (5a))
 *   d_workspace, bytes  caller-owned device memory, see above
 *   stream     hipStream_t (void*), used by every later call
 * On success *out owns host memory only; free it with dmr_destroy. */
int dmr_create(const dmr_params *p, const double *seed_base,
               const double *seed_fine, void *d_workspace, size_t bytes,
               void *stream, dmr_sim **out);

/* Release the handle (not the workspace).  Waits for queued work. */
void dmr_destroy(dmr_sim *s);

/* Queue n base (coarse) steps: per step the coarse EM update, two fine
 * substeps with boundary transfer and the fine -> coarse transfer
 * (Sec. III.C), every 1/8 period the window and continuity step on both
 * levels plus density transfers, and every regrid_every steps the growth
 * test (which synchronises the stream to read back 16 bytes of extents). */
int dmr_step(dmr_sim *s, int64_t n);

/* Run the growth test now (Sec. III.A-D); grows the patch if needed. */
int dmr_regrid(dmr_sim *s);

/* Patch extents in base cells {I0, J0, I1, J1}; all zero when there is no
 * patch.  For DMR_RULE_UNION: the bounding box of the active blocks, which
 * is also the region level-1 fields are read and written over (entries
 * outside the union are not part of the level and read 0).  Synchronises
 * the stream. */
int dmr_get_patch(dmr_sim *s, int32_t ext[4]);

/* DMR_RULE_UNION only (EINVAL otherwise).  dmr_get_blocks: the active blocks
 * of the fine level, [NBy][NBx] uint8 (1 = refined), NBx = nx/block;
 * synchronises the stream.  dmr_add_blocks: add the blocks set in mask
 * [NBy][NBx] to the fine level (growth only, Sec. III.D); entities new to the
 * level take Eq. (5a) values from the base level as in a growth; EINVAL if a
 * block lies within one block of the outer boundary or left of the source
 * line's margin.  Synchronises the stream. */
int dmr_get_blocks(dmr_sim *s, uint8_t *dst);
int dmr_add_blocks(dmr_sim *s, const uint8_t *mask);

/* Result of the last growth test: block flags [NBy][NBx] (uint8), their
 * exclusive prefix sum, the compacted list of flagged block ids (row-major
 * block index by*NBx+bx, ascending) and its length.  Any pointer may be
 * NULL; list must hold NBx*NBy entries.  Synchronises the stream. */
int dmr_get_regrid(dmr_sim *s, uint8_t *flags, int32_t *scan, int32_t *list,
                   int32_t *count);

/* Rows and columns of a field on a level (RING: 8*(ny+1) rows). */
int dmr_field_dims(dmr_sim *s, int field, int level, int32_t dims[2]);

/* Copy a field into dst (host or device memory, bytes >= rows*cols*4),
 * converted to SI.  Synchronises the stream. */
int dmr_read_field(dmr_sim *s, int field, int level, float *dst,
                   size_t bytes, int dst_on_device);

/* Overwrite a field (tests, fault injection, restarts); ERMS2 is read-only.
 * Synchronises the stream. */
int dmr_write_field(dmr_sim *s, int field, int level, const float *src,
                    size_t bytes, int src_on_device);

/* Simulated time (s) and base steps taken. */
int dmr_time(dmr_sim *s, double *t, int64_t *step);

/* Checkpoint and restart of the explicit time stepping (Sec. II.B, III.C: the
 * state at a base step is the fields of both levels, the density, the window
 * and the patch extents).  A saved state is a 256-byte header (format tag,
 * a hash of the parameters, step, window block count, patch) followed by the
 * live planes: base level Hz at n+1/2 and n-1/2, Ex, Ey, Jx, Jy, n, acc, the
 * 8 window slots; patch Hz, Ex, Ey, Jx, Jy, n, acc, 8 slots over the patch
 * rows of the full-domain fine grid; for DMR_RULE_UNION, then the block map
 * (one byte per block, padded to 256 bytes).
 *   dmr_state_bytes  bytes of a saved state of this handle (fixed by its
 *                    parameters).
 *   dmr_save         writes the state of the handle after all queued work
 *                    (synchronizes) to dst: host memory (dst_on_device = 0)
 *                    or device memory, 256-byte aligned; caller-owned.
 *   dmr_load         replaces the handle's state with one saved from a handle
 *                    created with the same parameters (EINVAL otherwise, and
 *                    for a buffer that is not a saved state); the next
 *                    dmr_step continues from the saved step.  A recorded
 *                    adjoint tape of the handle is invalidated.
 * ENOMEM if bytes is below dmr_state_bytes. */
int dmr_state_bytes(const dmr_sim *s, size_t *bytes);
int dmr_save(dmr_sim *s, void *dst, size_t bytes, int dst_on_device);
int dmr_load(dmr_sim *s, const void *src, size_t bytes, int src_on_device);

/* Wait for queued work; returns DMR_EUNSTABLE if a continuity step saw a
 * non-finite density or window value, DMR_EHIP on a HIP error. */
int dmr_sync(dmr_sim *s);

/* Per-kernel timing with HIP events on the handle's stream (off by
 * default).  Classes: 0 base-level EM step (with the patch substeps when
 * they run in the same launch), 1 fine EM substep, 2 continuity (both
 * levels), 3 growth test and prolongation.  One pair of events brackets
 * each run of consecutive launches of one class within a dmr_step call
 * (events between back-to-back launches would add their own latency to
 * each), so the time of a class is that of its launches and of the gaps
 * between them.  dmr_get_timing fills total milliseconds and launch counts
 * per class since the last reset and synchronises the stream. */
int dmr_set_timing(dmr_sim *s, int on);
int dmr_get_timing(dmr_sim *s, double ms[4], int64_t launches[4]);

/* Text of the last error on this handle (never NULL). */
const char *dmr_last_error(const dmr_sim *s);

/* ---- adjoint (reverse mode) ----------------------------------------------
 * Gradients of a linear functional of the final density,
 *   F = sum_nodes w_c n_c(t_final) + sum_nodes w_f n_f(t_final)
 * (e.g. the integral of n over a window: w = dx^2 on the window's nodes),
 * with respect to the incident amplitude E0 (Sec. II.B), the ionisation
 * coefficients A and beta of nu_i in Eq. (4), and the seed density, through
 * the whole refined update (Eqs. (1)-(5), Sec. III): the exact discrete
 * adjoint of the float32 forward, in float32 with float64 accumulation of
 * the scalar gradients.  The patch layout of the recorded run (its extents
 * at t = 0 and each growth) is held fixed: growth decisions are integer and
 * have no derivative, the Eq. (5a) prolongations they trigger are
 * differentiated.  Checkpoints every ckpt_every steps, recomputation of one
 * segment at a time (sqrt(N) checkpointing for ckpt_every ~ sqrt(steps)).
 *
 * Tape: caller-owned device memory (256-byte aligned) of
 * dmr_adjoint_tape_bytes; it holds the checkpoints (the coarse window planes
 * once, plus one per window block of the run), two segments of stored
 * forward values and the adjoint state, and must stay untouched between
 * dmr_forward_record and dmr_backward. */
int dmr_adjoint_tape_bytes(const dmr_params *p, int64_t steps, int ckpt_every,
                           size_t *bytes);

/* The tape for a run whose patch never spans more than fine_rows fine node
 * rows (r (J1 - J0) + 1 of the largest, i.e. the last, patch; <= 0: all
 * rows, as dmr_adjoint_tape_bytes).  The fine planes of the checkpoints and
 * of the stored steps hold only that many rows (the adjoint state still
 * spans the fine grid).  dmr_forward_record takes the rows from the size of
 * the tape it is given and fails with ENOMEM when the patch outgrows them
 * (the handle has then advanced: record again on a fresh one). */
int dmr_adjoint_tape_bytes_rows(const dmr_params *p, int64_t steps, int ckpt_every,
                                int32_t fine_rows, size_t *bytes);

/* Advance a fresh handle (t = 0) by `steps` base steps exactly as dmr_step
 * does, recording checkpoints and the patch history into the tape.
 * EINVAL if the handle has already stepped; ENOMEM if the tape is small
 * (for the current patch, or for a patch the run grows to). */
int dmr_forward_record(dmr_sim *s, int64_t steps, int ckpt_every, void *d_tape,
                       size_t bytes);

/* Reverse sweep over the recorded run.
 *   d_w_coarse  device float32 weights on the base nodes [ny+1][nx+1]
 *   d_w_fine    device float32 weights on the full-domain fine nodes
 *               [r*ny+1][r*nx+1] (entries outside the final patch unused),
 *               or NULL
 *   d_grad_seed       out, device float32 [ny+1][nx+1]: dF/d(base seed),
 *                     through the Eq. (5a) fine seed when the t = 0 patch
 *                     interpolated it; may be NULL
 *   d_grad_seed_fine  out, device float32 [r*ny+1][r*nx+1]: dF/d(fine
 *                     seed) when dmr_create was given one (else zeros); may
 *                     be NULL
 *   grad        out, host: dF/dE0 (per V/m of peak amplitude), dF/dA,
 *               dF/dbeta (A_ion and beta_ion of the power-law source; zero
 *               with the Townsend source, where they do not enter)
 * The handle is left at t_final, as after the record.  Synchronises. */
int dmr_backward(dmr_sim *s, const void *d_tape, const float *d_w_coarse,
                 const float *d_w_fine, float *d_grad_seed, float *d_grad_seed_fine,
                 double grad[3]);

/* sum over the nodes of a level (fine: full-domain grid) of w * n, with w
 * device float32 [rows][cols] of that grid; float64 sum in a fixed order.
 * Synchronises. */
int dmr_weighted_sum(dmr_sim *s, int level, const float *d_w, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * dmr_weighted_sum with its per-block partial sums (at most 1024) and the
 * result in a library-owned static device array (8 KB per GPU, held until
 * the process ends) instead of the handle's workspace; the same bits as
 * dmr_weighted_sum.  Every call on one GPU shares that array, so calls that
 * overlap on a GPU (any handle, any stream) race: serialise them.  EINVAL
 * for a level not present or more partial sums than the array holds (no
 * level reaches that: the partial count is capped at 1024), EHIP if the
 * array's address could not be found on the workspace's device.
 * Synchronises. */
int dmr_weighted_sum_static(dmr_sim *s, int level, const float *d_w, double *out);

/* ---- batched form -------------------------------------------------------
 * count independent simulations (grid sizes and physical parameters may
 * differ; steps per period, mode, continuity switch and regrid cadence must
 * agree) advanced in lockstep: each per-step kernel is one launch over the
 * tiles of all instances, the steps of every steady 256-step interval are
 * replayed from one captured HIP graph, and the streaming segment length,
 * load depth, fine tile height and subcycle schedule are chosen by timing
 * real steps (all choices give bit-identical results; choices are cached
 * per size key).
 * The batch runs on a private stream ordered after / before the caller's
 * stream with events.  Results per instance equal those of dmr_step on a
 * dmr_create'd simulation with the same inputs, bit for bit. */
typedef struct dmr_batch dmr_batch;

/* Workspace for count instances p[0..count-1] (instances + launch tables). */
int dmr_batch_workspace_bytes(const dmr_params *p, int count, size_t *bytes);

/* seed_base / seed_fine: arrays of count host pointers as in dmr_create (the
 * arrays themselves or any entry may be NULL). */
int dmr_batch_create(const dmr_params *p, int count, const double *const *seed_base,
                     const double *const *seed_fine, void *d_workspace, size_t bytes,
                     void *stream, dmr_batch **out);

/* Queue n base steps of every instance (growth tests every regrid_every). */
int dmr_batch_step(dmr_batch *b, int64_t n);

/* Borrowed handle of instance k for dmr_read_field, dmr_get_patch, dmr_time
 * and the like; do not dmr_step or dmr_destroy it. */
int dmr_batch_instance(dmr_batch *b, int k, dmr_sim **out);

/* Wait; DMR_EUNSTABLE if any instance saw a non-finite value. */
int dmr_batch_sync(dmr_batch *b);

/* Launch configuration {segment rows, load depth, fine tile rows, graph on,
 * subcycle schedule}.  Schedules (all give the same bits): 0 a base-level
 * launch and one launch per fine substep; 1 a base-level launch and one
 * launch of both substeps (temporally blocked; r = 4: two launches of two
 * substeps); 2 the base step and both substeps in one launch (r = 2).
 * Schedules 1 and 2 need rectangular patches (no union levels).  The batch
 * picks them by timing real steps of the run, per size key; set_config
 * forces one (and disables the timing-based choice); EINVAL for a schedule
 * the instances do not allow. */
int dmr_batch_config(dmr_batch *b, int32_t cfg[5]);
int dmr_batch_set_config(dmr_batch *b, const int32_t cfg[5]);

void dmr_batch_destroy(dmr_batch *b);
const char *dmr_batch_last_error(const dmr_batch *b);

#ifdef __cplusplus
}
#endif
#endif
