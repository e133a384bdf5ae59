// dmr_api.hip -- host side of the C ABI in include/dmr.h: parameter checks,
// derived coefficients, workspace carving, the subcycling schedule of
// Sec. III.C and the regrid cadence of Sec. III.D.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dmr.h"
#include "dmr_kernels.h"

#include <mutex>

// Scratch of the allocation-free entry point dmr_weighted_sum_static: the
// per-block partial sums of the weighted density sum (at most kStaticParts)
// and the result.  One copy per GPU, held until the process ends; host code
// uses the address hipGetSymbolAddress returns for the device, never the
// array's name.
constexpr int kStaticParts = 1024;
static __device__ __align__(256) double scratch[kStaticParts + 1];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// the array's address on device dev, looked up once per device with that
// device current (nullptr if the lookup failed)
double* static_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_tried[dev]) {
    g_scratch_tried[dev] = true;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[dev] = (double*)ptr;
    (void)hipGetLastError();
    if (cur != dev) (void)hipSetDevice(cur);
  }
  return g_scratch[dev];
}
}  // namespace

using namespace dmr;

namespace {

// CODATA 2018
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kKb = 1.380649e-23;  // J/K
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kPlanes = 21;  // Hz,Ex,Ey,Jx,Jy x2, n x2, acc, 8 window slots

struct Level {
  int NX = 0, NY = 0, pitch = 0;
  size_t plane = 0;
  float *hz[2] = {}, *ex[2] = {}, *ey[2] = {}, *jx[2] = {}, *jy[2] = {};
  float *n[2] = {}, *acc = nullptr, *ring = nullptr;
  float* hz_mid = nullptr;  // patch with r = 4: Hz after substep r/2
  double dx = 0, dt = 0;
  int spp = 0, spb = 0;
  float S = 0, c1 = 0, a = 0, kn = 0, cmur = 0;
};

size_t plane_floats(int NX, int NY, int* pitch) {
  const int p = (NX + 1 + 63) / 64 * 64;
  *pitch = p;
  const size_t n = (size_t)p * (NY + 1);
  return (n + 63) / 64 * 64;
}

struct Layout {
  size_t plane0 = 0, plane1 = 0;
  int pitch0 = 0, pitch1 = 0;
  size_t off_l1 = 0, off_flag = 0, off_scan = 0, off_list = 0, off_desc = 0,
         off_err = 0, off_stage = 0, total = 0;
  int NB = 0;
  // union-of-blocks fine level: two block maps, two tile lists (64 x 4 tiles
  // at most over the fine domain)
  size_t off_act = 0, off_tiles = 0, off_cfb = 0;
  size_t max_tiles = 0;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

bool refined(const dmr_params* p) { return p->mode != DMR_UNIFORM; }

Layout layout_of(const dmr_params* p) {
  Layout L;
  L.plane0 = plane_floats(p->nx, p->ny, &L.pitch0);
  size_t off = align256(L.plane0 * kPlanes * sizeof(float));
  L.off_l1 = off;
  size_t stage = L.plane0;
  if (refined(p)) {
    L.plane1 = plane_floats(p->r * p->nx, p->r * p->ny, &L.pitch1);
    off += align256(L.plane1 * (kPlanes + (p->r > 2 ? 1 : 0)) * sizeof(float));
    stage = L.plane1;
    L.NB = (p->nx / p->block) * (p->ny / p->block);
  }
  const size_t nb = (size_t)std::max(L.NB, 1);
  L.off_flag = off;  off += align256(nb);
  L.off_scan = off;  off += align256(nb * 4);
  L.off_list = off;  off += align256(nb * 4);
  L.off_desc = off;  off += 256;
  L.off_err = off;   off += 256;
  L.off_stage = off; off += align256(stage * sizeof(float));
  if (refined(p) && p->regrid_rule == DMR_RULE_UNION) {
    L.max_tiles = (size_t)((p->r * p->nx + 1 + kTX - 1) / kTX) * ((p->r * p->ny + 1 + 3) / 4);
    L.off_act = off;   off += 2 * align256(nb);
    L.off_tiles = off; off += 2 * align256(L.max_tiles * sizeof(int2));
    L.off_cfb = off;   off += align256(L.max_tiles * kCfbStride * sizeof(float));
  }
  L.total = off;
  return L;
}

int check_params(const dmr_params* p, std::string* why) {
  auto bad = [&](const char* m) { *why = m; return DMR_EINVAL; };
  if (!p) return bad("params is NULL");
  if (p->struct_size != sizeof(dmr_params)) return bad("struct_size mismatch");
  if (p->nx < 4 || p->ny < 4) return bad("nx, ny must be >= 4");
  // patch tiles address rows with 24-bit products of the byte pitch
  if ((long)p->nx * (p->r > 1 ? p->r : 1) >= (1L << 21))
    return bad("a level must be narrower than 2^21 cells");
  if (p->cells_per_lambda < 4) return bad("cells_per_lambda must be >= 4");
  if (!(p->courant > 0.0) || p->courant > 1.0 / std::sqrt(2.0) + 1e-12)
    return bad("Courant number must be in (0, 1/sqrt(2)] (2-D Yee stability)");
  const double sppd = p->cells_per_lambda / p->courant;
  const long spp = std::lround(sppd);
  if (std::fabs(sppd - spp) > 1e-9 || spp % kRing)
    return bad("cells_per_lambda/courant must be an integer multiple of 8");
  if (!(p->freq_hz > 0) || !(p->p_torr > 0)) return bad("freq_hz, p_torr > 0");
  if (!(p->fine_filter >= 0.0) || p->fine_filter > 1.0 / 64.0)
    return bad("fine_filter must be in [0, 1/64]");
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1)
    return bad("bc must be DMR_BC_MUR or DMR_BC_PEC");
  if (p->mode < 0 || p->mode > 2) return bad("bad mode");
  if (p->d_mode < 0 || p->d_mode > 1) return bad("bad d_mode");
  if (p->tfsf_i < 0 || p->tfsf_i >= p->nx) return bad("tfsf_i out of range");
  if (p->source_model < 0 || p->source_model > 1) return bad("bad source_model");
  if (p->source_model == DMR_SOURCE_TOWNSEND &&
      (!(p->A_town >= 0.0) || !(p->B_town > 0.0) || !(p->nu_att >= 0.0)))
    return bad("Townsend source needs A_town >= 0, B_town > 0, nu_att >= 0");
  if (!(p->beta_rec >= 0.0) || p->beta_rec > 2.0) return bad("beta_rec must be in [0, 2]");
  if (refined(p)) {
    if (p->r != 2 && p->r != 4) return bad("r must be 2 or 4");
    if (p->block < 2 || p->nx % p->block || p->ny % p->block)
      return bad("block must divide nx and ny");
    if (p->nx / p->block < 3 || p->ny / p->block < 3)
      return bad("need at least 3x3 blocks");
    if (p->mode == DMR_DYNAMIC &&
        (p->regrid_every <= 0 || p->regrid_every % (spp / kRing)))
      return bad("regrid_every must be a positive multiple of steps per window block");
    if (p->regrid_rule < 0 || p->regrid_rule > 2) return bad("bad regrid_rule");
    if (p->regrid_rule == DMR_RULE_UNION) {
      if (p->r != 2) return bad("the union-of-blocks fine level needs r = 2");
      if (p->block < 8 || (p->block & (p->block - 1)))
        return bad("the union-of-blocks fine level needs a power-of-two block >= 8");
      const int* e = p->static_ext;
      if (p->mode == DMR_STATIC &&
          (e[0] % p->block || e[1] % p->block || e[2] % p->block || e[3] % p->block))
        return bad("static_ext of the union-of-blocks fine level must be whole blocks");
    }
    if (p->mode == DMR_DYNAMIC && p->regrid_rule == DMR_RULE_LINES &&
        (p->m_lx < 1 || p->m_ly < 1 || p->m_ex < 1 || p->m_ey < 1 || !(p->n_line > 0.0)))
      return bad("the threshold-line rule needs m_lx, m_ly, m_ex, m_ey >= 1, n_line > 0");
    if (p->mode == DMR_STATIC) {
      const int* e = p->static_ext;
      if (e[0] < 1 || e[1] < 1 || e[2] > p->nx - 1 || e[3] > p->ny - 1 ||
          e[0] >= e[2] || e[1] >= e[3] || (p->tfsf_i > 0 && e[0] <= p->tfsf_i))
        return bad("static_ext outside the allowed region");
    }
  }
  return DMR_OK;
}

// Adjoint recording (the adjoint section below): what one replayed base step
// stores, and what it did.
struct StepStore {
  float *cexi, *ceyi, *cexp, *ceyp, *cn, *ce2;             // coarse
  float *fex0, *fey0, *fex1, *fey1, *fex2, *fey2, *fn, *fe2;  // patch
};
struct StepMeta {
  int has = 0, ext[4] = {0, 0, 0, 0};  // patch during the step
  int sync = 0, update = 0, slot = 0;  // window block closed after it
  int grow = 0, gnew[4] = {0, 0, 0, 0};  // growth after it
};
struct StepCtx {
  bool store = false;  // copy the step's forward values into ss
  bool last = false;   // last step of its segment (E after substep 2 is stored;
                       // otherwise it is the next step's stored E entering)
  StepStore ss{};
  bool forced = false;  // replay: apply force_ext instead of the growth test
  bool force_grow = false;
  int force_ext[4] = {0, 0, 0, 0};
  StepMeta meta;
};
struct Ckpt {
  int64_t step = 0, blocks = 0;
  int ccur = 0, ncur = 0, has = 0, ext[4] = {0, 0, 0, 0}, ty1 = 16;
};
struct Growth {
  int64_t after = 0;  // base steps completed when it happened
  int ext[4] = {0, 0, 0, 0};
};
struct AdjTape {
  char* base = nullptr;
  size_t bytes = 0;
  int64_t steps = 0;
  int every = 0, nck = 0;
  int frows = 0;  // fine node rows of each checkpoint / stored-step slot
  std::vector<Ckpt> ck;
  Ckpt fin;
  std::vector<Growth> grow;
  bool valid = false;
};

}  // namespace

struct dmr_sim {
  dmr_params p{};
  hipStream_t st = nullptr;
  int dev = -1;  // device holding the workspace
  Layout lay;
  char* ws = nullptr;
  std::string err = "";
  // derived scalars
  double omega = 0, lambda = 0, nu_m = 0, n_c = 0, eeff = 0, e0 = 0;
  double De = 0, Da = 0, n_amb = 0, ktil = 0, eta0 = 0;
  Level L0, L1;
  bool has_patch = false;
  int ext[4] = {0, 0, 0, 0};  // base cells
  int64_t step = 0, blocks = 0;
  int ccur = 0, ncur = 0;
  int seg0 = 16, depth0 = 2, ty1 = 16;
  // both patch substeps in one launch (dmr_step only; the adjoint's record and
  // replay and the batched form run them one launch each, bit-identically)
  bool fuse_fine = true;
  // base-level step and both patch substeps in one launch (dmr_step only)
  bool combine = true;
  long fuse_max = 1L << 20;  // fine cells up to which the two-substep launch is used
  // one-substep launches of large rectangular r = 2 patches: the streaming
  // form from stream_min fine cells on (DMR_FINE_STREAM=0/1 forces either).
  // Off by default: on config 2's 4.7 M-cell patch it takes 89.5 us per
  // substep against 87.8 us for the tile form
  long stream_min = LONG_MAX;
  int stream_force = -1;
  int fseg = 0, fdepth = 0;  // its rows per segment and load depth (0: by size)
  int nt1 = 1024;  // threads per patch tile
  // continuity of both levels in one launch (small rectangular r = 2 patch);
  // DMR_CONT_MERGE=0/1 forces either form
  int cont_merge = -1;
  int tw1 = 0;     // patch tile width of the combined step (0: by patch size)
  uint8_t* d_flag = nullptr;
  int32_t *d_scan = nullptr, *d_list = nullptr;
  int* d_desc = nullptr;
  int* d_err = nullptr;
  float* stage = nullptr;
  int h_desc[16] = {};
  // patch built at t = 0, and whether its density came from a fine seed
  bool had0 = false, keep_n0 = false;
  int ext0[4] = {0, 0, 0, 0};
  int peak[2] = {0, 0};  // base node of the seed's first maximum (row by row)
  // union-of-blocks fine level: block maps on the device (current d_act[acur],
  // the other one free for the next growth) and on the host, the tiles of
  // the level (d_tiles) and of the last growth (d_ptiles), 64 x tyu
  bool uni = false;
  uint8_t* d_act[2] = {nullptr, nullptr};
  int acur = 0;
  std::vector<uint8_t> h_act, h_act_new, h_flag;
  int2 *d_tiles = nullptr, *d_ptiles = nullptr;
  float* d_cfb = nullptr;  // Eq. (5b) values from substep 1 to substep 2, per tile
  std::vector<int2> h_tiles, h_ptiles;
  int ntiles = 0, tyu = 4;
  int64_t ugen = 0;  // growths of the level (the batch rebuilds its tables on a change)
  bool tyu_env = false;  // tile rows fixed by DMR_UTY
  AdjTape tape;
  hipStream_t rep_st = nullptr;  // the adjoint's replay stream (default priority)
  hipEvent_t ev_rep[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr}, ev_sync = nullptr;
  // timing
  bool timing = false;
  // a group of consecutive launches of one class, bracketed by one pair of
  // events (events between back-to-back launches would add their own
  // latency to every launch)
  struct Ev { int cls; int n; hipEvent_t a, b; };
  bool ev_open = false;  // the last group has no end event yet
  std::vector<Ev> evs;
  size_t ev_used = 0;
  double t_ms[4] = {0, 0, 0, 0};
  int64_t t_n[4] = {0, 0, 0, 0};
};

namespace {

int fail(dmr_sim* s, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (s) s->err = buf;
  return code;
}

int hipfail(dmr_sim* s, hipError_t e, const char* what) {
  return fail(s, DMR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(s, call)                              \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hipfail(s, e_, #call); \
  } while (0)

void derive(dmr_sim* s) {
  const dmr_params& p = s->p;
  s->omega = 2.0 * kPi * p.freq_hz;
  s->lambda = kC0 / p.freq_hz;
  s->nu_m = 5.3e9 * p.p_torr;  // Sec. II.A
  s->n_c = kMe * kEps0 * s->omega * s->omega / (kQe * kQe);
  s->eeff = 1.0 / (1.0 + (s->omega / s->nu_m) * (s->omega / s->nu_m));
  const double e_cr = p.ecr_over_p * 100.0 * p.p_torr;
  const double e_bd = e_cr * std::sqrt(1.0 + (s->omega / s->nu_m) * (s->omega / s->nu_m));
  s->e0 = std::sqrt(2.0) * p.erms_over_ebd * e_bd;
  s->De = kQe * p.te_ev / (kMe * s->nu_m);
  s->Da = p.mu_i_760 * (760.0 / p.p_torr) * (p.te_ev + p.ti_ev);
  s->n_amb = kEps0 * p.te_ev / (kQe * p.L_amb * p.L_amb);
  s->eta0 = kC0 / (kEps0 * kC0 * kC0);  // mu0 c with mu0 = 1/(eps0 c^2)
}

void level_coeffs(dmr_sim* s, Level* L, double dx, double dt, int spp) {
  L->dx = dx;
  L->dt = dt;
  L->spp = spp;
  L->spb = spp / kRing;
  const double S = kC0 * dt / dx;
  const double a = std::exp(-s->nu_m * dt);
  const double b = kQe * kQe * (1.0 - a) / (kMe * s->nu_m);
  L->S = (float)S;
  L->a = (float)a;
  L->c1 = (float)(0.5 * (1.0 + a));
  L->kn = (float)(dt * b / (4.0 * kEps0));
  L->cmur = (float)((S - 1.0) / (S + 1.0));
}

// the base level's step sizes and coefficients and the incident wavenumber;
// no device memory is touched
void setup_scalars(dmr_sim* s) {
  const dmr_params& p = s->p;
  derive(s);
  const double dx0 = s->lambda / p.cells_per_lambda;
  const double dt0 = p.courant * dx0 / kC0;
  const int spp0 = (int)std::lround(p.cells_per_lambda / p.courant);
  // numerical wavenumber of the 1-D Yee wave
  s->ktil = 2.0 / dx0 * std::asin(std::sin(0.5 * s->omega * dt0) / p.courant);
  level_coeffs(s, &s->L0, dx0, dt0, spp0);
}

void carve(dmr_sim* s, Level* L, size_t off, size_t plane, int pitch, int NX,
           int NY) {
  float* base = (float*)(s->ws + off);
  L->NX = NX;
  L->NY = NY;
  L->pitch = pitch;
  L->plane = plane;
  float* q = base;
  for (int b = 0; b < 2; b++) {
    L->hz[b] = q; q += plane;
    L->ex[b] = q; q += plane;
    L->ey[b] = q; q += plane;
    L->jx[b] = q; q += plane;
    L->jy[b] = q; q += plane;
    L->n[b] = q;  q += plane;
  }
  L->acc = q; q += plane;
  L->ring = q;
  L->hz_mid = q + (size_t)kRing * plane;  // allocated for the r = 4 patch only
}

// incident Ey at (x, t): E0 g(t - x/c) sin(w t - k~ x), sin^2 ramp g
double ey_inc(const dmr_sim* s, double x, double t) {
  const double tr = s->p.ramp_periods / s->p.freq_hz;
  const double tau = t - x / kC0;
  double g = 1.0;
  if (tau <= 0.0) g = 0.0;
  else if (tau < tr) { const double q = std::sin(0.5 * kPi * tau / tr); g = q * q; }
  return s->e0 * g * std::sin(s->omega * t - s->ktil * x);
}

void harvest(dmr_sim* s);

// close the open group of launches (its end event after the last launch)
void ev_close(dmr_sim* s) {
  if (!s->ev_open) return;
  (void)hipEventRecord(s->evs[s->ev_used].b, s->st);
  s->ev_open = false;
  s->ev_used++;
  if (s->ev_used >= 4096) harvest(s);
}

// a launch of class cls follows: extend the open group if it is of the same
// class, else start a new group
void ev_begin(dmr_sim* s, int cls) {
  if (!s->timing) return;
  if (s->ev_open && s->evs[s->ev_used].cls == cls) {
    s->evs[s->ev_used].n++;
    return;
  }
  ev_close(s);
  if (s->ev_used == s->evs.size()) {
    dmr_sim::Ev e{cls, 0, nullptr, nullptr};
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
    s->evs.push_back(e);
  }
  s->evs[s->ev_used].cls = cls;
  s->evs[s->ev_used].n = 1;
  (void)hipEventRecord(s->evs[s->ev_used].a, s->st);
  s->ev_open = true;
}

void harvest(dmr_sim* s) {
  ev_close(s);
  if (!s->ev_used) return;
  (void)hipStreamSynchronize(s->st);
  for (size_t k = 0; k < s->ev_used; k++) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->evs[k].a, s->evs[k].b) == hipSuccess) {
      s->t_ms[s->evs[k].cls] += ms;
      s->t_n[s->evs[k].cls] += s->evs[k].n;
    }
  }
  s->ev_used = 0;
}

// after a launch: groups of the step classes stay open for the next launch
// of the same class; the growth test (class 3) waits on the host between its
// launches, so its groups end at once
void ev_end(dmr_sim* s) {
  if (s->timing && s->ev_open && s->evs[s->ev_used].cls == 3) ev_close(s);
}

// rows per segment of the streaming base kernel: long segments for
// bandwidth, short ones when the grid is too small to fill the chip
int stream_rows(int NX, int NY) {
  if (const char* e = getenv("DMR_SEG")) {
    const int v = atoi(e);
    if (v >= 2) return v;
  }
  // a wave walks its rows one memory round trip (over the load depth) apart:
  // small grids take short segments and many waves
  // (measured: 8 rows on 4096x2048, 16 on 8192x4096, 2 on config-1 sizes)
  const long waves_x = (NX + 1 + 61) / 62;
  int seg = 16;
  while (seg > 2 && waves_x * ((NY + seg) / seg) < 16384) seg >>= 1;
  return seg;
}

// rows in flight per wave (measured on 512x256 ... 4096x2048: 2 for
// segments of up to 4 rows and for long ones, 4 in between)
int stream_depth(int seg) {
  if (const char* e = getenv("DMR_DEPTH")) return atoi(e) >= 4 ? 4 : 2;
  return (seg >= 8 && seg <= 16) ? 4 : 2;
}

// the streaming form of the one-substep patch launch: large rectangular
// r = 2 patches outside the adjoint's replay (the replay copies values
// around the tile kernel)
bool stream_patch(const dmr_sim* s, long fine_cells) {
  if (s->uni || s->p.r != 2) return false;
  if (s->stream_force >= 0) return s->stream_force == 1;
  return fine_cells >= s->stream_min;
}

// rows per segment of the streaming patch substep: every segment re-reads
// five rows of E around its start, so segments are longer than the base
// kernel's; halve them only while the grid has too few waves to fill the chip
int fine_stream_rows(int NX, int NY) {
  const long waves_x = (NX + 1 + 57) / 58;
  int seg = 32;
  while (seg > 8 && waves_x * ((NY + seg) / seg) < 8192) seg >>= 1;
  return seg;
}

int tile_rows(int NX, int NY) {
  if (const char* e = getenv("DMR_TY")) {
    const int v = atoi(e);
    if (v == 4 || v == 8 || v == 16) return v;
  }
  // enough tiles to cover the 256 compute units several times over
  const long tiles16 = (long)((NX + kTX) / kTX) * ((NY + 16) / 16);
  if (tiles16 >= 2048) return 16;
  const long tiles8 = (long)((NX + kTX) / kTX) * ((NY + 8) / 8);
  if (tiles8 >= 1024) return 8;
  return 4;
}

int prolong(dmr_sim* s, const int ne[4], bool keep_n) {
  Level &C = s->L0, &F = s->L1;
  const int r = s->p.r;
  ProlongArgs A{};
  A.L = r * ne[0]; A.B = r * ne[1]; A.R = r * ne[2]; A.T = r * ne[3];
  if (s->has_patch) {
    A.oL = r * s->ext[0]; A.oB = r * s->ext[1];
    A.oR = r * s->ext[2]; A.oT = r * s->ext[3];
  }
  A.pitch = F.pitch; A.cpitch = C.pitch;
  A.plane = F.plane; A.cplane = C.plane;
  A.keep_n = keep_n ? 1 : 0;
  A.rf = r;
  const int c = s->ccur;
  A.chz = C.hz[c]; A.chz_prev = C.hz[1 - c];
  A.cex = C.ex[c]; A.cey = C.ey[c]; A.cjx = C.jx[c]; A.cjy = C.jy[c];
  A.cn = C.n[s->ncur]; A.cacc = C.acc; A.cring = C.ring;
  A.hz = F.hz[0]; A.ex = F.ex[0]; A.ey = F.ey[0]; A.jx = F.jx[0]; A.jy = F.jy[0];
  A.n = F.n[s->ncur]; A.acc = F.acc; A.ring = F.ring;
  ev_begin(s, 3);
  hipError_t e = launch_prolong(A, s->st);
  ev_end(s);
  if (e != hipSuccess) return hipfail(s, e, "prolongation launch");
  for (int k = 0; k < 4; k++) s->ext[k] = ne[k];
  s->has_patch = true;
  const int fw = r * (ne[2] - ne[0]), fh = r * (ne[3] - ne[1]);
  s->ty1 = tile_rows(fw, fh);

  return DMR_OK;
}

// Growth by the threshold lines of Sec. III.D: the patch sides are the lines;
// a side whose line carries a node with n > n_line moves out by m_ex (x) or
// m_ey (y).  The first patch is m_lx x m_ly cells centred on the seed peak.
int regrid_lines(dmr_sim* s, bool keep_n) {
  const dmr_params& p = s->p;
  const int Bk = p.block;
  int xmin = 1;
  if (p.tfsf_i > 0) xmin = std::max(xmin, (p.tfsf_i + 2 * Bk - 1) / Bk);
  int ne[4];
  if (!s->has_patch) {
    ne[0] = s->peak[0] - p.m_lx / 2;
    ne[1] = s->peak[1] - p.m_ly / 2;
    ne[2] = ne[0] + p.m_lx;
    ne[3] = ne[1] + p.m_ly;
  } else {
    int* f = (int*)s->stage;
    ev_begin(s, 3);
    hipError_t e = launch_line_flags(s->L0.n[s->ncur], s->L0.pitch, s->ext[0], s->ext[1],
                                     s->ext[2], s->ext[3], (float)p.n_line, f, s->st);
    ev_end(s);
    if (e != hipSuccess) return hipfail(s, e, "threshold-line launch");
    int h[4];
    HIPCHK(s, hipMemcpyAsync(h, f, sizeof(h), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (int q = 0; q < 4; q++) ne[q] = s->ext[q];
    if (h[0]) ne[0] -= p.m_ex;
    if (h[1]) ne[2] += p.m_ex;
    if (h[2]) ne[1] -= p.m_ey;
    if (h[3]) ne[3] += p.m_ey;
  }
  ne[0] = std::max(ne[0], xmin * Bk);
  ne[1] = std::max(ne[1], Bk);
  ne[2] = std::min(ne[2], p.nx - Bk);
  ne[3] = std::min(ne[3], p.ny - Bk);
  if (ne[0] >= ne[2] || ne[1] >= ne[3]) return DMR_OK;  // no room for a patch
  if (s->has_patch && !memcmp(ne, s->ext, sizeof(ne))) return DMR_OK;
  return prolong(s, ne, keep_n);
}

// ---- the fine level as a union of blocks ----------------------------------
// The blocks the growth test flags (Sec. III.A/B) are refined as they are,
// instead of their bounding box: the level is every cell of an active block
// (r = 2, blocks of 2^fbs fine cells a side), with the edges and nodes
// touching them.  Tiles (64 x tyu fine nodes) run where a cell of their
// one-cell dilation is active; growth prolongs only what is new.

// first block column a fine region may use: one block clear of the outer
// boundary and of the source line
int block_xmin(const dmr_params& p) {
  int xmin = 1;
  if (p.tfsf_i > 0) xmin = std::max(xmin, (p.tfsf_i + 2 * p.block - 1) / p.block);
  return xmin;
}

int log2i(int v) {
  int k = 0;
  while ((1 << k) < v) k++;
  return k;
}

// tiles whose dilated cells [i0-1, i0+63] x [j0-1, j0+ty-1] meet a block
// with pick(block) set
template <class Pick>
void union_tiles(const dmr_sim* s, int ty, Pick pick, std::vector<int2>* out) {
  const dmr_params& p = s->p;
  const int fnx = p.r * p.nx, fny = p.r * p.ny, FB = p.r * p.block;
  const int NBx = p.nx / p.block, NBy = p.ny / p.block;
  const int ntx = (fnx + 1 + kTX - 1) / kTX, nty = (fny + 1 + ty - 1) / ty;
  out->clear();
  for (int ty_ = 0; ty_ < nty; ty_++) {
    const int jl = std::max(ty_ * ty - 1, 0), jh = std::min(ty_ * ty + ty - 1, fny - 1);
    if (jl > jh) continue;
    for (int tx = 0; tx < ntx; tx++) {
      const int il = std::max(tx * kTX - 1, 0), ih = std::min(tx * kTX + kTX - 1, fnx - 1);
      if (il > ih) continue;
      bool hit = false;
      for (int bj = jl / FB; bj <= std::min(jh / FB, NBy - 1) && !hit; bj++)
        for (int bi = il / FB; bi <= std::min(ih / FB, NBx - 1) && !hit; bi++)
          hit = pick(bj * NBx + bi);
      if (hit) out->push_back(make_int2(tx, ty_));
    }
  }
}

void union_level_args(const dmr_sim* s, int* fbs, int* nbkx, int* nbky) {
  *fbs = log2i(s->p.r * s->p.block);
  *nbkx = s->p.nx / s->p.block;
  *nbky = s->p.ny / s->p.block;
}

// tile rows: short tiles (more of them, shorter per-tile chains) while the
// level is small (measured on config 2: 33.1 ms with 4 rows against 36.0 ms
// with 16 for 256 coarse steps), the tile_rows rule once it is large
void pick_union_rows(dmr_sim* s, const std::vector<uint8_t>& map) {
  if (s->tyu_env) return;
  long act = 0;
  for (uint8_t v : map) act += v;
  const long fb = (long)s->p.r * s->p.block;
  const long cells = act * fb * fb;
  s->tyu = cells / (kTX * 16) >= 2048 ? 16 : cells / (kTX * 8) >= 1024 ? 8 : 4;
}

// extents (bounding box of the active blocks) and presence of the level
void union_extents(dmr_sim* s) {
  const dmr_params& p = s->p;
  const int NBx = p.nx / p.block, NBy = p.ny / p.block;
  int bx0 = NBx, by0 = NBy, bx1 = 0, by1 = 0;
  for (int b = 0; b < NBx * NBy; b++)
    if (s->h_act[b]) {
      bx0 = std::min(bx0, b % NBx); by0 = std::min(by0, b / NBx);
      bx1 = std::max(bx1, b % NBx + 1); by1 = std::max(by1, b / NBx + 1);
    }
  s->has_patch = bx1 > bx0;
  if (!s->has_patch) bx0 = by0 = bx1 = by1 = 0;
  s->ext[0] = bx0 * p.block; s->ext[1] = by0 * p.block;
  s->ext[2] = bx1 * p.block; s->ext[3] = by1 * p.block;
}

// make h_act the level as it stands (restart): map and tile list to the
// device, extents; no prolongation (the state carries the fine data)
int union_install(dmr_sim* s) {
  pick_union_rows(s, s->h_act);
  union_tiles(s, s->tyu, [&](int b) { return s->h_act[b] != 0; }, &s->h_tiles);
  HIPCHK(s, hipMemcpyAsync(s->d_act[s->acur], s->h_act.data(), s->h_act.size(),
                           hipMemcpyHostToDevice, s->st));
  if (!s->h_tiles.empty())
    HIPCHK(s, hipMemcpyAsync(s->d_tiles, s->h_tiles.data(), s->h_tiles.size() * sizeof(int2),
                             hipMemcpyHostToDevice, s->st));
  s->ntiles = (int)s->h_tiles.size();
  union_extents(s);
  HIPCHK(s, hipStreamSynchronize(s->st));
  return DMR_OK;
}

// Add the blocks of add ([NBy][NBx]) to the level.  strict: a block outside
// the margins is an error (else it is left out).
int grow_union(dmr_sim* s, const uint8_t* add, bool keep_n, bool strict) {
  const dmr_params& p = s->p;
  const int NBx = p.nx / p.block, NBy = p.ny / p.block, xmin = block_xmin(p);
  auto inside = [&](int b) {
    const int bx = b % NBx, by = b / NBx;
    return bx >= xmin && by >= 1 && bx <= NBx - 2 && by <= NBy - 2;
  };
  s->h_act_new = s->h_act;
  bool changed = false;
  for (int b = 0; b < NBx * NBy; b++) {
    if (!add[b]) continue;
    if (!inside(b)) {
      if (strict) return fail(s, DMR_EINVAL, "block %d outside the margins", b);
      continue;
    }
    if (!s->h_act_new[b]) { s->h_act_new[b] = 1; changed = true; }
  }
  if (!changed) return DMR_OK;
  pick_union_rows(s, s->h_act_new);
  const std::vector<uint8_t>& nw = s->h_act_new;
  const std::vector<uint8_t>& od = s->h_act;
  union_tiles(s, s->tyu, [&](int b) { return nw[b] && !od[b]; }, &s->h_ptiles);
  union_tiles(s, s->tyu, [&](int b) { return nw[b] != 0; }, &s->h_tiles);
  uint8_t* act_new = s->d_act[1 - s->acur];
  HIPCHK(s, hipMemcpyAsync(act_new, nw.data(), nw.size(), hipMemcpyHostToDevice, s->st));
  HIPCHK(s, hipMemcpyAsync(s->d_ptiles, s->h_ptiles.data(), s->h_ptiles.size() * sizeof(int2),
                           hipMemcpyHostToDevice, s->st));
  HIPCHK(s, hipMemcpyAsync(s->d_tiles, s->h_tiles.data(), s->h_tiles.size() * sizeof(int2),
                           hipMemcpyHostToDevice, s->st));
  Level &C = s->L0, &F = s->L1;
  ProlongArgs A{};
  A.L = 0; A.B = 0; A.R = F.NX; A.T = F.NY;
  A.pitch = F.pitch; A.cpitch = C.pitch;
  A.plane = F.plane; A.cplane = C.plane;
  A.keep_n = keep_n ? 1 : 0;
  A.rf = p.r;
  const int c = s->ccur;
  A.chz = C.hz[c]; A.chz_prev = C.hz[1 - c];
  A.cex = C.ex[c]; A.cey = C.ey[c]; A.cjx = C.jx[c]; A.cjy = C.jy[c];
  A.cn = C.n[s->ncur]; A.cacc = C.acc; A.cring = C.ring;
  A.hz = F.hz[0]; A.ex = F.ex[0]; A.ey = F.ey[0]; A.jx = F.jx[0]; A.jy = F.jy[0];
  A.n = F.n[s->ncur]; A.acc = F.acc; A.ring = F.ring;
  A.act = act_new; A.act_old = s->d_act[s->acur];
  A.seed = keep_n ? s->stage : nullptr;  // the fine seed, uploaded there at creation
  union_level_args(s, &A.fbs, &A.nbkx, &A.nbky);
  ev_begin(s, 3);
  hipError_t e = launch_prolong_union(A, s->d_ptiles, (int)s->h_ptiles.size(), s->tyu, s->st);
  ev_end(s);
  if (e != hipSuccess) return hipfail(s, e, "prolongation launch");
  s->acur = 1 - s->acur;
  s->h_act.swap(s->h_act_new);
  s->ntiles = (int)s->h_tiles.size();
  s->ugen++;
  union_extents(s);
  return DMR_OK;
}

// the growth test of the union: the flagged blocks inside the margins join
int regrid_union(dmr_sim* s, bool keep_n) {
  const dmr_params& p = s->p;
  const int Bk = p.block, NBx = p.nx / Bk, NBy = p.ny / Bk;
  int* D = s->h_desc;
  for (int k = 0; k < 16; k++) D[k] = 0;
  D[10] = block_xmin(p); D[11] = 1; D[12] = NBx - 1; D[13] = NBy - 1;
  HIPCHK(s, hipMemcpyAsync(s->d_desc, D, 16 * sizeof(int), hipMemcpyHostToDevice, s->st));
  FlagArgs F{};
  F.n = s->L0.n[s->ncur];
  F.pitch = s->L0.pitch; F.NX = p.nx; F.NY = p.ny; F.Bk = Bk;
  F.NBx = NBx; F.NBy = NBy;
  F.thr = (float)(p.n_thr_over_nc * s->n_c);
  F.flo = (float)(p.n_floor_over_nc * s->n_c);
  F.g2 = (float)(p.grad_thr * p.grad_thr);
  F.bflag = s->d_flag;
  ScanArgs S{};
  S.bflag = s->d_flag; S.NB = NBx * NBy; S.NBx = NBx; S.NBy = NBy;
  S.scan = s->d_scan; S.list = s->d_list; S.desc = s->d_desc;
  ev_begin(s, 3);
  hipError_t e = launch_regrid_test(F, S, s->st);
  ev_end(s);
  if (e != hipSuccess) return hipfail(s, e, "regrid launch");
  s->h_flag.assign((size_t)NBx * NBy, 0);
  HIPCHK(s, hipMemcpyAsync(s->h_flag.data(), s->d_flag, s->h_flag.size(),
                           hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  return grow_union(s, s->h_flag.data(), keep_n, false);
}

int regrid(dmr_sim* s, bool keep_n) {
  const dmr_params& p = s->p;
  if (p.regrid_rule == DMR_RULE_UNION) return regrid_union(s, keep_n);
  if (p.regrid_rule == DMR_RULE_LINES) return regrid_lines(s, keep_n);
  const int Bk = p.block, NBx = p.nx / Bk, NBy = p.ny / Bk;
  int* D = s->h_desc;
  for (int k = 0; k < 4; k++) D[k] = s->has_patch ? s->ext[k] / Bk : 0;
  // margins: one block clear of the outer boundary and of the source line
  int xmin = 1;
  if (p.tfsf_i > 0) xmin = std::max(xmin, (p.tfsf_i + 2 * Bk - 1) / Bk);
  D[10] = xmin; D[11] = 1; D[12] = NBx - 1; D[13] = NBy - 1;
  HIPCHK(s, hipMemcpyAsync(s->d_desc, D, 16 * sizeof(int), hipMemcpyHostToDevice, s->st));
  FlagArgs F{};
  F.n = s->L0.n[s->ncur];
  F.pitch = s->L0.pitch; F.NX = p.nx; F.NY = p.ny; F.Bk = Bk;
  F.NBx = NBx; F.NBy = NBy;
  F.thr = (float)(p.n_thr_over_nc * s->n_c);
  F.flo = (float)(p.n_floor_over_nc * s->n_c);
  F.g2 = (float)(p.grad_thr * p.grad_thr);
  F.bflag = s->d_flag;
  ScanArgs S{};
  S.bflag = s->d_flag; S.NB = NBx * NBy; S.NBx = NBx; S.NBy = NBy;
  S.scan = s->d_scan; S.list = s->d_list; S.desc = s->d_desc;
  ev_begin(s, 3);
  hipError_t e = launch_regrid_test(F, S, s->st);
  ev_end(s);
  if (e != hipSuccess) return hipfail(s, e, "regrid launch");
  HIPCHK(s, hipMemcpyAsync(D, s->d_desc, 16 * sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  if (!D[9]) return DMR_OK;
  const int ne[4] = {D[4] * Bk, D[5] * Bk, D[6] * Bk, D[7] * Bk};
  if (ne[2] <= ne[0]) return DMR_OK;
  return prolong(s, ne, keep_n);
}

void em_args_level(EMArgs* A, const Level& L, int src, int dst, const float* n,
                   float* acc) {
  A->hz0 = L.hz[src]; A->ex0 = L.ex[src]; A->ey0 = L.ey[src];
  A->jx0 = L.jx[src]; A->jy0 = L.jy[src];
  A->hz1 = L.hz[dst]; A->ex1 = L.ex[dst]; A->ey1 = L.ey[dst];
  A->jx1 = L.jx[dst]; A->jy1 = L.jy[dst];
  A->n = n; A->acc = acc;
  A->pitch = L.pitch;
  A->S = L.S; A->c1 = L.c1; A->a = L.a; A->kn = L.kn; A->cmur = L.cmur;
}

int stream_blocks_x(int NX) { return ((NX + 1 + 61) / 62 + kThreads / 64 - 1) / (kThreads / 64); }

// argument blocks of the four per-step launches, for buffer parities c
// (E/H/J) and nc (density); shared by the plain and the batched schedules
void make_base_em(const dmr_sim* s, int c, int nc, EMArgs* A) {
  const Level& C = s->L0;
  const dmr_params& p = s->p;
  *A = EMArgs{};
  em_args_level(A, C, c, 1 - c, C.n[nc], C.acc);
  A->L = 0; A->B = 0; A->R = p.nx; A->T = p.ny;
  A->bc_x = p.bc_x; A->bc_y = p.bc_y;
  A->is = p.tfsf_i;
  A->seg = s->seg0;
  A->nseg = stream_segments(p.ny, s->seg0);
  A->nbx = stream_blocks_x(p.nx);
}

void incident_values(const dmr_sim* s, int64_t step, float* ey, float* hz) {
  const Level& C = s->L0;
  *ey = *hz = 0.f;
  if (s->p.tfsf_i <= 0) return;
  const double t = (double)step * C.dt, xs = s->p.tfsf_i * C.dx;
  *ey = (float)ey_inc(s, xs, t);
  *hz = (float)ey_inc(s, xs - 0.5 * C.dx, t + 0.5 * C.dt);
}

void make_fine_em(const dmr_sim* s, int m, int c, int nc, int ty, EMArgs* G) {
  const Level &C = s->L0, &F = s->L1;
  const dmr_params& p = s->p;
  const int r = p.r;
  *G = EMArgs{};
  const int src = (m - 1) & 1, dst = m & 1;
  em_args_level(G, F, src, dst, F.n[nc], F.acc);
  G->L = r * s->ext[0]; G->B = r * s->ext[1];
  G->R = r * s->ext[2]; G->T = r * s->ext[3];
  G->cex0 = C.ex[c]; G->cey0 = C.ey[c];
  G->cex1 = C.ex[1 - c]; G->cey1 = C.ey[1 - c];
  G->cpitch = C.pitch;
  G->frac = (float)m / (float)r;
  G->gamma = (float)p.fine_filter;
  G->rf = r;
  if (r > 2 && m == r / 2) G->hz_save = F.hz_mid;
  if (r > 2 && m == r) G->hz_lo = F.hz_mid;
  if (m == r) {
    G->restrict_on = 1;
    G->chz = C.hz[1 - c]; G->cex = C.ex[1 - c]; G->cey = C.ey[1 - c];
    G->cjx = C.jx[1 - c]; G->cjy = C.jy[1 - c];
  }
  G->nbx = (G->R - G->L + 1 + kTX - 1) / kTX;
  if (s->uni) {  // the whole fine domain; membership from the block map
    G->L = 0; G->B = 0; G->R = F.NX; G->T = F.NY;
    G->act = s->d_act[s->acur];
    union_level_args(s, &G->fbs, &G->nbkx, &G->nbky);
    G->cnx = p.nx; G->cny = p.ny;
    G->utiles = s->d_tiles;
    // Eq. (5b) values handed from substep 1 to the last substep
    if (m == 1) G->cfb_next = s->d_cfb;
    if (m == r) G->cfb_prev = s->d_cfb;
  }
  (void)ty;
}

// recombination coefficient of Eq. (4), m^3/s: beta 1e-13 (300 K / T_e)^(1/2)
double rei_of(const dmr_params& p) {
  if (!(p.beta_rec > 0.0)) return 0.0;
  const double te_k = p.te_ev * kQe / kKb;
  return p.beta_rec * 1e-13 * std::sqrt(300.0 / te_k);
}

void make_base_cont(const dmr_sim* s, int nc, ContArgs* K) {
  const Level& C = s->L0;
  const dmr_params& p = s->p;
  *K = ContArgs{};
  K->n0 = C.n[nc]; K->n1 = C.n[1 - nc];
  K->acc = C.acc; K->ring = C.ring; K->plane = C.plane; K->pitch = C.pitch;
  K->L = 0; K->B = 0; K->R = p.nx; K->T = p.ny;
  K->inv_spp = (float)(1.0 / C.spp);
  K->dtn = (float)(C.spb * C.dt);
  K->inv_dx2 = (float)(1.0 / (C.dx * C.dx));
  K->eeff_p2 = (float)(s->eeff / (1.0e4 * p.p_torr * p.p_torr));
  K->half_beta = (float)(0.5 * p.beta_ion);
  K->att = (float)std::pow(p.ecr_over_p, p.beta_ion);
  K->nuA = (float)(s->nu_m * p.A_ion);
  if (p.source_model == DMR_SOURCE_TOWNSEND) {
    // gamma v_d = [100 A_town p exp(-B_town / y)] [mu_e 100 p y], y = E_eff/(100 p)
    const double mu_e = kQe / (kMe * s->nu_m);
    K->town = 1;
    K->tK = (float)(1.0e4 * p.A_town * p.p_torr * p.p_torr * mu_e);
    K->tB = (float)p.B_town;
    K->tatt = (float)p.nu_att;
  }
  K->rei = (float)rei_of(p);
  K->inv_namb = (float)(1.0 / s->n_amb);
  K->De = (float)s->De; K->Da = (float)s->Da;
  K->d_const_mode = p.d_mode == DMR_D_CONST;
  K->d_const = (float)p.d_const;
  K->err = s->d_err;
  K->nbx = (p.nx + 1 + kTX - 1) / kTX;
}

void make_fine_cont(const dmr_sim* s, int nc, ContArgs* G) {
  const Level &C = s->L0, &F = s->L1;
  const dmr_params& p = s->p;
  make_base_cont(s, nc, G);
  G->n0 = F.n[nc]; G->n1 = F.n[1 - nc];
  G->acc = F.acc; G->ring = F.ring; G->plane = F.plane; G->pitch = F.pitch;
  G->L = p.r * s->ext[0]; G->B = p.r * s->ext[1];
  G->R = p.r * s->ext[2]; G->T = p.r * s->ext[3];
  G->inv_spp = (float)(1.0 / F.spp);
  G->dtn = (float)(F.spb * F.dt);
  G->inv_dx2 = (float)(1.0 / (F.dx * F.dx));
  G->cn1 = C.n[1 - nc]; G->cpitch = C.pitch;
  G->rf = p.r;
  G->nbx = (G->R - G->L + 1 + kTX - 1) / kTX;
  if (s->uni) {
    G->L = 0; G->B = 0; G->R = F.NX; G->T = F.NY;
    G->act = s->d_act[s->acur];
    union_level_args(s, &G->fbs, &G->nbkx, &G->nbky);
    G->utiles = s->d_tiles;
  }
}

// copy jobs of one stored plane: whole coarse planes, patch rows of fine ones
void job(CopyJobs* J, const float* src, float* dst, size_t n) {
  J->job[J->count++] = CopyJob{src, dst, n};
}

void job_rows(CopyJobs* J, const dmr_sim* s, const float* src, float* dst) {
  const Level& F = s->L1;
  const size_t off = (size_t)(s->p.r * s->ext[1]) * F.pitch;
  const size_t n = (size_t)(s->p.r * (s->ext[3] - s->ext[1]) + 1) * F.pitch;
  job(J, src + off, dst + off, n);
}

int run_copies(dmr_sim* s, const CopyJobs& J) {
  const hipError_t e = launch_copy(J, s->st);
  return e == hipSuccess ? DMR_OK : hipfail(s, e, "tape copy");
}

// One base step with subcycling (Sec. III.C), the window/continuity cadence
// and the regrid cadence.  With cx, the step also reports what it did and,
// for the adjoint's replay, stores its forward values and applies a
// recorded growth instead of running the growth test.
int base_step(dmr_sim* s, StepCtx* cx = nullptr) {
  const dmr_params& p = s->p;
  const int c = s->ccur;
  const bool st = cx && cx->store;
  if (cx) {
    cx->meta = StepMeta{};
    cx->meta.has = s->has_patch;
    for (int q = 0; q < 4; q++) cx->meta.ext[q] = s->ext[q];
  }
  // the two-substep tile keeps a 7-cell halo in LDS (one block per CU): it
  // wins where the patch is small and the step latency-bound; large patches
  // stream better as two one-substep launches
  const long fine_cells =
      s->has_patch ? (long)p.r * p.r * (s->ext[2] - s->ext[0]) * (s->ext[3] - s->ext[1]) : 0;
  const bool big = fine_cells > s->fuse_max;
  const bool fuse = s->has_patch && s->fuse_fine && !big && !s->uni;
  // replay: the fused kernels store the step's values themselves; the
  // one-substep form takes copies
  const bool kst = st && (!s->has_patch || fuse);
  if (st && !kst) {
    CopyJobs J{};
    const size_t n0 = s->L0.plane;
    job(&J, s->L0.ex[c], cx->ss.cexi, n0);
    job(&J, s->L0.ey[c], cx->ss.ceyi, n0);
    job(&J, s->L0.n[s->ncur], cx->ss.cn, n0);
    if (s->has_patch) {
      job_rows(&J, s, s->L1.ex[0], cx->ss.fex0);
      job_rows(&J, s, s->L1.ey[0], cx->ss.fey0);
      job_rows(&J, s, s->L1.n[s->ncur], cx->ss.fn);
    }
    if (int rc = run_copies(s, J)) return rc;
  }
  // coarse (or uniform) EM step n -> n+1
  EMArgs A;
  make_base_em(s, c, s->ncur, &A);
  incident_values(s, s->step, &A.ey_src, &A.hz_src);
  hipError_t e = hipSuccess;
  if (kst) {
    A.stix = cx->ss.cexi; A.stiy = cx->ss.ceyi;
    A.stox = cx->ss.cexp; A.stoy = cx->ss.ceyp; A.stn = cx->ss.cn;
  }
  auto fine_stores = [&](EMArgs* G) {
    if (!kst) return;
    G->st0x = cx->ss.fex0; G->st0y = cx->ss.fey0;
    G->st1x = cx->ss.fex1; G->st1y = cx->ss.fey1;
    G->st2x = cx->last ? cx->ss.fex2 : nullptr;
    G->st2y = cx->last ? cx->ss.fey2 : nullptr;
    G->stn = cx->ss.fn;
  };
  // the fused forms are bit-identical to the separate launches.  r = 4
  // (4-row tiles, no replay): the launch takes the base step and substeps
  // (1, 2); (3, 4) and the fine -> coarse transfer follow in a launch of
  // their own, so the base waves store every coarse entity
  const bool r4 = p.r == 4;
  const bool combined = fuse && s->combine && (!r4 || (s->ty1 == 4 && !kst));
  // what patch tiles need to form the coarse E after the base step on their
  // boundary lines themselves: the coarse state entering the step
  auto coarse_state = [&](EMArgs* G) {
    const Level& C = s->L0;
    G->chz0 = C.hz[c]; G->cjx0 = C.jx[c]; G->cjy0 = C.jy[c]; G->cn0 = C.n[s->ncur];
    G->cS = C.S; G->cc1 = C.c1; G->ckn = C.kn; G->cis = p.tfsf_i;
    G->cey_src = A.ey_src; G->chz_src = A.hz_src;
    G->cnx = p.nx; G->cny = p.ny;
  };
  if (combined) {  // base step and both patch substeps (r = 4: the first pair), one launch
    Level& F = s->L1;
    A.skip_on = r4 ? 0 : 1;
    A.sL = s->ext[0]; A.sB = s->ext[1]; A.sR = s->ext[2]; A.sT = s->ext[3];
    EMArgs G;
    make_fine_em(s, r4 ? 2 : p.r, c, s->ncur, s->ty1, &G);  // r = 2: restriction targets
    em_args_level(&G, F, 0, 1, F.n[s->ncur], F.acc);
    G.frac = 1.f / (float)p.r;  // time fraction of substep 1
    if (r4) {  // as the first pair of the two-launch r = 4 form
      G.hz_save = nullptr;
      G.hz_lo = nullptr;
    }
    coarse_state(&G);
    fine_stores(&G);
    ev_begin(s, 0);
    e = launch_dmr_step(A, G, s->seg0, s->depth0, s->ty1, s->tw1, s->st, r4);
    ev_end(s);
    if (e != hipSuccess) return hipfail(s, e, "combined step launch");
    if (!r4) {  // r = 4: the second pair writes buffer 0 again
      std::swap(F.hz[0], F.hz[1]);
      std::swap(F.ex[0], F.ex[1]);
      std::swap(F.ey[0], F.ey[1]);
      std::swap(F.jx[0], F.jx[1]);
      std::swap(F.jy[0], F.jy[1]);
    }
  } else {
    ev_begin(s, 0);
    e = launch_em_stream(A, s->seg0, s->depth0, s->st);
    ev_end(s);
    if (e != hipSuccess) return hipfail(s, e, "base EM launch");
  }
  if (st && !kst && !s->has_patch) {  // with a patch: stored after substep 1
    CopyJobs J{};
    job(&J, s->L0.ex[1 - c], cx->ss.cexp, s->L0.plane);
    job(&J, s->L0.ey[1 - c], cx->ss.ceyp, s->L0.plane);
    if (int rc = run_copies(s, J)) return rc;
  }
  if (combined && !r4) {
    // done above
  } else if (fuse && p.r == 4) {  // substeps (1, 2) then (3, 4), one launch each
    Level& F = s->L1;
    for (int h = combined ? 1 : 0; h < 2; h++) {
      EMArgs G;
      make_fine_em(s, 2 * h + 2, c, s->ncur, s->ty1, &G);  // the second pair restricts
      em_args_level(&G, F, h, 1 - h, F.n[s->ncur], F.acc);
      G.frac = (float)(2 * h + 1) / (float)p.r;  // time fraction of the pair's first
      G.hz_save = nullptr;
      G.hz_lo = nullptr;
      ev_begin(s, 1);
      if (combined) {  // the frame tile of the combined launch, for the second pair
        coarse_state(&G);
        e = launch_fine2_fast(G, s->tw1, s->st);
      } else {
        e = launch_fine2(G, s->ty1, s->nt1, s->st);
      }
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "fine EM launch");
    }
  } else if (fuse) {  // both substeps, one launch
    Level& F = s->L1;
    EMArgs G;
    make_fine_em(s, p.r, c, s->ncur, s->ty1, &G);  // restriction targets
    em_args_level(&G, F, 0, 1, F.n[s->ncur], F.acc);
    G.frac = 1.f / (float)p.r;  // time fraction of substep 1
    fine_stores(&G);
    ev_begin(s, 1);
    if (s->ty1 == 4 && !kst) {  // 4-row tiles: the frame tile of the combined step
      coarse_state(&G);
      e = launch_fine2_fast(G, s->tw1, s->st);
    } else {
      e = launch_fine2(G, s->ty1, s->nt1, s->st);
    }
    ev_end(s);
    if (e != hipSuccess) return hipfail(s, e, "fine EM launch");
    // the new state is in buffer 1: make it buffer 0
    std::swap(F.hz[0], F.hz[1]);
    std::swap(F.ex[0], F.ex[1]);
    std::swap(F.ey[0], F.ey[1]);
    std::swap(F.jx[0], F.jx[1]);
    std::swap(F.jy[0], F.jy[1]);
  } else if (s->has_patch) {  // two fine substeps (Sec. III.C)
    for (int m = 1; m <= p.r; m++) {
      EMArgs G;
      make_fine_em(s, m, c, s->ncur, s->ty1, &G);
      ev_begin(s, 1);
      if (s->uni) {
        e = launch_em_union(G, s->d_tiles, s->ntiles, s->tyu, s->nt1, s->st);
      } else if (stream_patch(s, fine_cells)) {
        const int sg = s->fseg > 0 ? s->fseg : fine_stream_rows(G.R - G.L, G.T - G.B);
        e = launch_fine_stream(G, sg, s->fdepth > 0 ? s->fdepth : 2, s->st);
      } else {
        e = launch_em(G, true, s->ty1, s->nt1, s->st);
      }
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "fine EM launch");
      if (st && (m == 1 || cx->last)) {
        CopyJobs J{};
        job_rows(&J, s, s->L1.ex[m & 1], m == 1 ? cx->ss.fex1 : cx->ss.fex2);
        job_rows(&J, s, s->L1.ey[m & 1], m == 1 ? cx->ss.fey1 : cx->ss.fey2);
        if (m == 1) {  // the coarse E after the coarse step (the transfer comes in substep 2)
          job(&J, s->L0.ex[1 - c], cx->ss.cexp, s->L0.plane);
          job(&J, s->L0.ey[1 - c], cx->ss.ceyp, s->L0.plane);
        }
        if (int rc = run_copies(s, J)) return rc;
      }
    }
  }
  s->ccur = 1 - c;
  s->step++;
  if (p.continuity_on && s->step % s->L0.spb == 0) {
    const int slot = (int)(s->blocks % kRing);
    s->blocks++;
    const int update = s->blocks >= kRing;
    if (cx) {
      cx->meta.sync = 1;
      cx->meta.update = update;
      cx->meta.slot = slot;
    }
    ContArgs K;
    make_base_cont(s, s->ncur, &K);
    K.slot = slot; K.update = update;
    // a small rectangular r = 2 patch on a small (latency-bound) grid: both
    // levels in one launch (its boundary lines take one block of their own;
    // measured: 5.7 instead of 9.3 us on 512 x 256, even on 1024 x 512,
    // slower on 4096 x 2048, where the coarse level streams better in the
    // plain launch)
    const long perim = s->has_patch ? 2L * p.r * ((s->ext[2] - s->ext[0]) + (s->ext[3] - s->ext[1])) : 0;
    const bool merge = s->has_patch && !s->uni && (p.r == 2 || p.r == 4) && perim <= 2048 &&
                       s->ext[2] > s->ext[0] && s->ext[3] > s->ext[1] &&
                       (s->cont_merge >= 0 ? s->cont_merge == 1 : (long)p.nx * p.ny <= (1L << 19));
    if (merge) {
      ContArgs G;
      make_fine_cont(s, s->ncur, &G);
      G.slot = slot; G.update = update;
      K.pL = s->ext[0]; K.pB = s->ext[1]; K.pR = s->ext[2]; K.pT = s->ext[3];
      ev_begin(s, 2);
      e = launch_cont2(K, G, s->st);
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "continuity launch");
    } else {
      ev_begin(s, 2);
      e = launch_cont(K, false, s->st);
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "continuity launch");
    }
    if (s->has_patch && !merge) {
      ContArgs G;
      make_fine_cont(s, s->ncur, &G);
      G.slot = slot; G.update = update;
      ev_begin(s, 2);
      if (s->uni) e = launch_cont_union(G, s->d_tiles, s->ntiles, s->tyu, s->st);
      else e = launch_cont(G, true, s->st);
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "fine continuity launch");
    }
    if (st && update) {  // the E_rms^2 each continuity step used
      const Level& C = s->L0;
      e = launch_ring_e2(C.ring, C.plane, C.pitch, 0, 0, p.nx, p.ny, cx->ss.ce2, s->st);
      if (e == hipSuccess && s->has_patch) {
        const Level& F = s->L1;
        const int r = p.r;
        e = launch_ring_e2(F.ring, F.plane, F.pitch, r * s->ext[0], r * s->ext[1],
                           r * s->ext[2], r * s->ext[3], cx->ss.fe2, s->st);
      }
      if (e != hipSuccess) return hipfail(s, e, "window sum launch");
    }
    if (update) s->ncur = 1 - s->ncur;
  }
  if (p.mode == DMR_DYNAMIC && s->step % p.regrid_every == 0) {
    if (cx && cx->forced) {
      if (!cx->force_grow) return DMR_OK;
      if (int rc = prolong(s, cx->force_ext, false)) return rc;
    } else {
      const bool had = s->has_patch;
      int before[4];
      for (int q = 0; q < 4; q++) before[q] = s->ext[q];
      if (int rc = regrid(s, false)) return rc;
      bool grew = s->has_patch != had;
      for (int q = 0; q < 4; q++) grew = grew || s->ext[q] != before[q];
      if (!grew || !cx) return DMR_OK;
    }
    cx->meta.grow = 1;
    for (int q = 0; q < 4; q++) cx->meta.gnew[q] = s->ext[q];
  }
  return DMR_OK;
}

struct View {
  const Level* L;
  int i0, j0, nx, ny;  // region origin and cells
};

int view_of(dmr_sim* s, int level, View* v) {
  if (level == 0) {
    *v = View{&s->L0, 0, 0, s->p.nx, s->p.ny};
    return DMR_OK;
  }
  if (level == 1 && s->has_patch) {
    const int r = s->p.r;
    *v = View{&s->L1, r * s->ext[0], r * s->ext[1], r * (s->ext[2] - s->ext[0]),
              r * (s->ext[3] - s->ext[1])};
    return DMR_OK;
  }
  return fail(s, DMR_EINVAL, "level %d not present", level);
}

int dims_of(int field, const View& v, int* rows, int* cols) {
  switch (field) {
  case DMR_HZ: *rows = v.ny; *cols = v.nx; return DMR_OK;
  case DMR_EX: case DMR_JX: *rows = v.ny + 1; *cols = v.nx; return DMR_OK;
  case DMR_EY: case DMR_JY: *rows = v.ny; *cols = v.nx + 1; return DMR_OK;
  case DMR_N: case DMR_ACC: case DMR_ERMS2:
    *rows = v.ny + 1; *cols = v.nx + 1; return DMR_OK;
  case DMR_RING: *rows = kRing * (v.ny + 1); *cols = v.nx + 1; return DMR_OK;
  }
  return DMR_EINVAL;
}

// device array and SI scale of a field (value_SI = scale * stored)
float* array_of(dmr_sim* s, int field, int level, double* scale) {
  Level& L = level == 0 ? s->L0 : s->L1;
  const int b = level == 0 ? s->ccur : 0;
  *scale = 1.0;
  switch (field) {
  case DMR_HZ: *scale = 1.0 / s->eta0; return L.hz[b];
  case DMR_EX: return L.ex[b];
  case DMR_EY: return L.ey[b];
  case DMR_JX: *scale = kEps0 / L.dt; return L.jx[b];
  case DMR_JY: *scale = kEps0 / L.dt; return L.jy[b];
  case DMR_N: return L.n[s->ncur];
  case DMR_ACC: return L.acc;
  case DMR_RING: return L.ring;
  }
  return nullptr;
}

}  // namespace

extern "C" {

int dmr_derived(const dmr_params* p, double* out, int n_out) {
  std::string why;
  const int rc = check_params(p, &why);
  if (rc) {
    fprintf(stderr, "dmr_derived: %s\n", why.c_str());
    return rc;
  }
  if (!out || n_out < 0) return DMR_EINVAL;
  dmr_sim* s = new (std::nothrow) dmr_sim();
  if (!s) return DMR_ENOMEM;
  s->p = *p;
  setup_scalars(s);
  ContArgs K;
  make_base_cont(s, 0, &K);
  const Level& L = s->L0;
  const double v[17] = {
      s->omega, s->lambda, L.dx, L.dt, s->nu_m, s->n_c, s->eeff,
      s->e0 / (std::sqrt(2.0) * p->erms_over_ebd), s->e0, s->De, s->Da, s->n_amb,
      (double)L.a, (double)L.kn * 4.0 * kEps0 / L.dt, s->ktil,
      (double)K.nuA * (double)K.att, (double)L.spp};
  for (int k = 0; k < n_out && k < 17; k++) out[k] = v[k];
  delete s;
  return DMR_OK;
}

int dmr_workspace_bytes(const dmr_params* p, size_t* bytes) {
  std::string why;
  const int rc = check_params(p, &why);
  if (rc) return rc;
  if (!bytes) return DMR_EINVAL;
  *bytes = layout_of(p).total;
  return DMR_OK;
}

int dmr_create(const dmr_params* p, const double* seed_base,
               const double* seed_fine, void* d_workspace, size_t bytes,
               void* stream, dmr_sim** out) {
  if (!out) return DMR_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = check_params(p, &why);
  if (rc) {
    fprintf(stderr, "dmr_create: %s\n", why.c_str());
    return rc;
  }
  const Layout lay = layout_of(p);
  if (!d_workspace || bytes < lay.total) return DMR_ENOMEM;
  dmr_sim* s = new (std::nothrow) dmr_sim();
  if (!s) return DMR_ENOMEM;
  s->p = *p;
  s->st = (hipStream_t)stream;
  s->lay = lay;
  s->ws = (char*)d_workspace;
  {
    // the device that holds the workspace; set up the static scratch array's
    // address there once (used only by dmr_weighted_sum_static)
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, d_workspace) == hipSuccess) s->dev = a.device;
    (void)hipGetLastError();
    if (s->dev >= 0) (void)static_scratch(s->dev);
  }
  setup_scalars(s);
  const double dx0 = s->L0.dx, dt0 = s->L0.dt;
  const int spp0 = s->L0.spp;
  carve(s, &s->L0, 0, lay.plane0, lay.pitch0, p->nx, p->ny);
  if (refined(p)) {
    carve(s, &s->L1, lay.off_l1, lay.plane1, lay.pitch1, p->r * p->nx, p->r * p->ny);
    level_coeffs(s, &s->L1, dx0 / p->r, dt0 / p->r, spp0 * p->r);
  }
  s->d_flag = (uint8_t*)(s->ws + lay.off_flag);
  s->d_scan = (int32_t*)(s->ws + lay.off_scan);
  s->d_list = (int32_t*)(s->ws + lay.off_list);
  s->d_desc = (int*)(s->ws + lay.off_desc);
  s->d_err = (int*)(s->ws + lay.off_err);
  s->stage = (float*)(s->ws + lay.off_stage);
  if (refined(p) && p->regrid_rule == DMR_RULE_UNION) {
    s->uni = true;
    const size_t nb = (size_t)lay.NB;
    s->d_act[0] = (uint8_t*)(s->ws + lay.off_act);
    s->d_act[1] = s->d_act[0] + align256(nb);
    s->d_tiles = (int2*)(s->ws + lay.off_tiles);
    s->d_ptiles = s->d_tiles + align256(lay.max_tiles * sizeof(int2)) / sizeof(int2);
    s->d_cfb = (float*)(s->ws + lay.off_cfb);
    s->h_act.assign(nb, 0);
    if (const char* f = getenv("DMR_UTY")) {
      const int v = atoi(f);
      if (v == 4 || v == 8 || v == 16) { s->tyu = v; s->tyu_env = true; }
    }
  }
  s->seg0 = stream_rows(p->nx, p->ny);
  if (const char* f = getenv("DMR_FUSE")) s->fuse_fine = atoi(f) != 0;
  // one launch per coarse step pays off where launch latency dominates; on
  // bandwidth-bound grids the base kernel's own launch shape is faster
  s->combine = (long)p->nx * p->ny <= (1L << 21);
  if (const char* f = getenv("DMR_COMBINE")) s->combine = atoi(f) != 0;
  // r = 2: the base step and both substeps in one launch; r = 4: the base
  // step and the first pair of substeps (4-row tiles), then the second pair
  if (const char* f = getenv("DMR_FUSE_MAX")) s->fuse_max = atol(f);
  if (const char* f = getenv("DMR_FNT")) s->nt1 = atoi(f) >= 1024 ? 1024 : 256;
  if (const char* f = getenv("DMR_TW")) { const int v = atoi(f); s->tw1 = (v == 16 || v == 32 || v == 64) ? v : 0; }
  if (const char* f = getenv("DMR_FINE_STREAM")) s->stream_force = atoi(f) != 0 ? 1 : 0;
  if (const char* f = getenv("DMR_CONT_MERGE")) s->cont_merge = atoi(f) != 0 ? 1 : 0;
  if (const char* f = getenv("DMR_FINE_SEG")) s->fseg = atoi(f) >= 2 ? atoi(f) : 0;
  if (const char* f = getenv("DMR_FINE_DEPTH")) s->fdepth = atoi(f) >= 4 ? 4 : 2;
  s->depth0 = stream_depth(s->seg0);
  hipError_t e = hipMemsetAsync(s->ws, 0, lay.total, s->st);
  if (e != hipSuccess) { rc = hipfail(s, e, "workspace clear"); delete s; return rc; }
  // seeds: float32 on the pitched node grid
  std::vector<float> h;
  auto upload = [&](const double* src, const Level& L, float* dst) -> hipError_t {
    h.assign(L.plane, 0.f);
    for (int j = 0; j <= L.NY; j++)
      for (int i = 0; i <= L.NX; i++)
        h[(size_t)j * L.pitch + i] = (float)src[(size_t)j * (L.NX + 1) + i];
    hipError_t r1 = hipMemcpyAsync(dst, h.data(), L.plane * sizeof(float),
                                   hipMemcpyHostToDevice, s->st);
    if (r1 != hipSuccess) return r1;
    return hipStreamSynchronize(s->st);
  };
  if (seed_base) {  // the seed's peak (the threshold-line rule centres the first patch on it)
    double best = seed_base[0];
    for (int j = 0; j <= p->ny; j++)
      for (int i = 0; i <= p->nx; i++)
        if (seed_base[(size_t)j * (p->nx + 1) + i] > best) {
          best = seed_base[(size_t)j * (p->nx + 1) + i];
          s->peak[0] = i; s->peak[1] = j;
        }
  }
  if (seed_base && (e = upload(seed_base, s->L0, s->L0.n[0])) != hipSuccess) {
    rc = hipfail(s, e, "seed upload");
    delete s;
    return rc;
  }
  const bool keep_n = refined(p) && seed_fine;
  // the union of blocks takes the fine seed on its own nodes only (through
  // the prolongation, from the staging plane); the patch keeps it in place
  if (keep_n && (e = upload(seed_fine, s->L1, s->uni ? s->stage : s->L1.n[0])) != hipSuccess) {
    rc = hipfail(s, e, "fine seed upload");
    delete s;
    return rc;
  }
  if (p->mode == DMR_STATIC && s->uni) {  // the blocks of static_ext
    const int Bk = p->block, NBx = p->nx / Bk;
    std::vector<uint8_t> add((size_t)lay.NB, 0);
    for (int by = p->static_ext[1] / Bk; by < p->static_ext[3] / Bk; by++)
      for (int bx = p->static_ext[0] / Bk; bx < p->static_ext[2] / Bk; bx++)
        add[(size_t)by * NBx + bx] = 1;
    rc = grow_union(s, add.data(), keep_n, true);
  } else if (p->mode == DMR_STATIC) {
    rc = prolong(s, p->static_ext, keep_n);
  } else if (p->mode == DMR_DYNAMIC) {
    rc = regrid(s, keep_n);
  }
  s->had0 = s->has_patch;
  s->keep_n0 = keep_n;
  for (int k = 0; k < 4; k++) s->ext0[k] = s->ext[k];
  if (!rc) {
    e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) rc = hipfail(s, e, "create");
  }
  if (rc) {
    fprintf(stderr, "dmr_create: %s\n", s->err.c_str());
    delete s;
    return rc;
  }
  *out = s;
  return DMR_OK;
}

void dmr_destroy(dmr_sim* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  if (s->rep_st) {
    (void)hipStreamSynchronize(s->rep_st);
    (void)hipStreamDestroy(s->rep_st);
    for (int b = 0; b < 2; b++) {
      (void)hipEventDestroy(s->ev_rep[b]);
      (void)hipEventDestroy(s->ev_adj[b]);
    }
    (void)hipEventDestroy(s->ev_sync);
  }
  for (auto& e : s->evs) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  delete s;
}

int dmr_step(dmr_sim* s, int64_t n) {
  if (!s || n < 0) return fail(s, DMR_EINVAL, "bad step count");
  for (int64_t k = 0; k < n; k++) {
    const int rc = base_step(s);
    if (rc) { ev_close(s); return rc; }
  }
  ev_close(s);  // a timing group does not span calls (the caller may queue other work)
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hipfail(s, e, "step");
  return DMR_OK;
}

int dmr_regrid(dmr_sim* s) {
  if (!s) return DMR_EINVAL;
  if (s->p.mode == DMR_UNIFORM) return fail(s, DMR_EINVAL, "uniform mode has no patch");
  return regrid(s, false);
}

int dmr_get_patch(dmr_sim* s, int32_t ext[4]) {
  if (!s || !ext) return DMR_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->st));
  for (int k = 0; k < 4; k++) ext[k] = s->has_patch ? s->ext[k] : 0;
  return DMR_OK;
}

int dmr_get_blocks(dmr_sim* s, uint8_t* dst) {
  if (!s || !dst) return DMR_EINVAL;
  if (!s->uni) return fail(s, DMR_EINVAL, "not a union-of-blocks fine level");
  HIPCHK(s, hipStreamSynchronize(s->st));
  memcpy(dst, s->h_act.data(), s->h_act.size());
  return DMR_OK;
}

int dmr_add_blocks(dmr_sim* s, const uint8_t* mask) {
  if (!s || !mask) return DMR_EINVAL;
  if (!s->uni) return fail(s, DMR_EINVAL, "not a union-of-blocks fine level");
  const int rc = grow_union(s, mask, false, true);
  if (rc) return rc;
  HIPCHK(s, hipStreamSynchronize(s->st));
  return DMR_OK;
}

int dmr_get_regrid(dmr_sim* s, uint8_t* flags, int32_t* scan, int32_t* list,
                   int32_t* count) {
  if (!s) return DMR_EINVAL;
  if (s->p.mode == DMR_UNIFORM) return fail(s, DMR_EINVAL, "uniform mode has no regrid");
  const size_t nb = (size_t)s->lay.NB;
  HIPCHK(s, hipStreamSynchronize(s->st));
  int cnt = 0;
  HIPCHK(s, hipMemcpy(&cnt, s->d_desc + 8, sizeof(int), hipMemcpyDeviceToHost));
  if (flags) HIPCHK(s, hipMemcpy(flags, s->d_flag, nb, hipMemcpyDeviceToHost));
  if (scan) HIPCHK(s, hipMemcpy(scan, s->d_scan, nb * 4, hipMemcpyDeviceToHost));
  if (list && cnt) HIPCHK(s, hipMemcpy(list, s->d_list, (size_t)cnt * 4, hipMemcpyDeviceToHost));
  if (count) *count = cnt;
  return DMR_OK;
}

int dmr_field_dims(dmr_sim* s, int field, int level, int32_t dims[2]) {
  if (!s || !dims) return DMR_EINVAL;
  View v;
  int rc = view_of(s, level, &v);
  if (rc) return rc;
  int rows, cols;
  if (dims_of(field, v, &rows, &cols)) return fail(s, DMR_EINVAL, "bad field %d", field);
  dims[0] = rows;
  dims[1] = cols;
  return DMR_OK;
}

int dmr_read_field(dmr_sim* s, int field, int level, float* dst, size_t bytes,
                   int dst_on_device) {
  if (!s || !dst) return DMR_EINVAL;
  View v;
  int rc = view_of(s, level, &v);
  if (rc) return rc;
  int rows, cols;
  if (dims_of(field, v, &rows, &cols)) return fail(s, DMR_EINVAL, "bad field %d", field);
  if (bytes < (size_t)rows * cols * sizeof(float)) return fail(s, DMR_EINVAL, "dst too small");
  const Level& L = *v.L;
  const int planes = field == DMR_RING ? kRing : 1;
  const int prow = rows / planes;
  for (int k = 0; k < planes; k++) {
    float* out = dst_on_device ? dst + (size_t)k * prow * cols : s->stage;
    hipError_t e;
    if (field == DMR_ERMS2) {
      e = launch_ring_sum(L.ring, L.plane, L.pitch, v.i0, v.j0, cols, prow, out, s->st);
    } else {
      double sc;
      const float* src = array_of(s, field, level, &sc);
      if (field == DMR_RING) src += (size_t)k * L.plane;
      e = launch_gather(src, L.pitch, v.i0, v.j0, cols, prow, (float)sc, out, s->st);
    }
    if (e != hipSuccess) return hipfail(s, e, "read launch");
    if (!dst_on_device)
      HIPCHK(s, hipMemcpyAsync(dst + (size_t)k * prow * cols, out,
                               (size_t)prow * cols * sizeof(float),
                               hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
  }
  return DMR_OK;
}

int dmr_write_field(dmr_sim* s, int field, int level, const float* src,
                    size_t bytes, int src_on_device) {
  if (!s || !src) return DMR_EINVAL;
  if (field == DMR_ERMS2) return fail(s, DMR_EINVAL, "ERMS2 is read-only");
  View v;
  int rc = view_of(s, level, &v);
  if (rc) return rc;
  int rows, cols;
  if (dims_of(field, v, &rows, &cols)) return fail(s, DMR_EINVAL, "bad field %d", field);
  if (bytes < (size_t)rows * cols * sizeof(float)) return fail(s, DMR_EINVAL, "src too small");
  const Level& L = *v.L;
  const int planes = field == DMR_RING ? kRing : 1;
  const int prow = rows / planes;
  double sc;
  float* arr = array_of(s, field, level, &sc);
  for (int k = 0; k < planes; k++) {
    const float* in = src + (size_t)k * prow * cols;
    if (!src_on_device) {
      HIPCHK(s, hipMemcpyAsync(s->stage, in, (size_t)prow * cols * sizeof(float),
                               hipMemcpyHostToDevice, s->st));
      in = s->stage;
    }
    float* a = arr + (field == DMR_RING ? (size_t)k * L.plane : 0);
    hipError_t e = launch_scatter(in, cols, prow, (float)(1.0 / sc), a, L.pitch,
                                  v.i0, v.j0, s->st);
    if (e != hipSuccess) return hipfail(s, e, "write launch");
    HIPCHK(s, hipStreamSynchronize(s->st));
  }
  return DMR_OK;
}

int dmr_time(dmr_sim* s, double* t, int64_t* step) {
  if (!s) return DMR_EINVAL;
  if (t) *t = (double)s->step * s->L0.dt;
  if (step) *step = s->step;
  return DMR_OK;
}

int dmr_sync(dmr_sim* s) {
  if (!s) return DMR_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->st));
  int flags[64];
  HIPCHK(s, hipMemcpy(flags, s->d_err, sizeof(flags), hipMemcpyDeviceToHost));
  for (int k = 0; k < 64; k++)
    if (flags[k]) return fail(s, DMR_EUNSTABLE, "non-finite density or window value");
  return DMR_OK;
}

int dmr_set_timing(dmr_sim* s, int on) {
  if (!s) return DMR_EINVAL;
  harvest(s);
  s->timing = on != 0;
  for (int k = 0; k < 4; k++) { s->t_ms[k] = 0; s->t_n[k] = 0; }
  return DMR_OK;
}

int dmr_get_timing(dmr_sim* s, double ms[4], int64_t launches[4]) {
  if (!s) return DMR_EINVAL;
  harvest(s);
  for (int k = 0; k < 4; k++) {
    if (ms) ms[k] = s->t_ms[k];
    if (launches) launches[k] = s->t_n[k];
  }
  return DMR_OK;
}

const char* dmr_last_error(const dmr_sim* s) {
  return s ? s->err.c_str() : "no handle";
}

}  // extern "C"

// ===========================================================================
// Adjoint: reverse mode of a recorded run.  dmr_forward_record advances the
// simulation from t = 0 like dmr_step, keeping a checkpoint of the state
// every ckpt_every base steps and the patch history.  dmr_backward walks the
// checkpoint segments from the last to the first: it restores the segment's
// checkpoint, replays its steps (same kernels, recorded growths applied
// instead of the growth test) storing the values the adjoint kernels need,
// then runs the adjoint of each step in reverse order.  Memory: checkpoints
// plus one segment of stored steps (sqrt(N) checkpointing when ckpt_every is
// about sqrt(steps)).
// ===========================================================================
namespace {

constexpr int kAdjPlanes = 26;       // lam state + temporaries per level
// planes of the live state (coarse: Hz, Hz of the other half level, E, J, n,
// acc, the kRing window planes; patch: Hz, E, J, n, acc, its window planes).
// A tape checkpoint leaves out the coarse window planes: the tape logs each
// window block's coarse plane once (the ring at a checkpoint is rebuilt from
// that log and the ring at the start of the recording).
constexpr int kLiveC = 8 + kRing, kCkF = 15;
constexpr int kCkC = 8;  // coarse planes per tape checkpoint
constexpr int kStC = 4, kStF = 4;    // planes stored per replayed step (E in, E out)
constexpr int kBkC = 2, kBkF = 2;    // per window block of a segment (n, E_rms^2)

struct TapeLayout {
  size_t adj_c = 0, adj_f = 0, ck = 0, ck_size = 0, store = 0, st_size = 0, src = 0,
         src_size = 0, u = 0, part = 0, part_per_step = 0, gsum = 0, wpart = 0, total = 0;
  // a bank of stored steps: `every` step slots, then nbk window-block slots
  // (the density is constant between continuity steps, E_rms^2 is taken at
  // them), then the patch E after the last substep of the segment's last step
  size_t bk_size = 0, last_size = 0, bank_size = 0;
  int nbk = 0;
  // the coarse window planes at the start of the recording, and one coarse
  // window plane per block closed during it
  size_t ring0 = 0, rlog = 0;
  int nlog = 0;
  int nck = 0;
  int frows = 0;      // fine node rows a checkpoint / stored-step slot holds
  size_t fplane = 0;  // floats of one fine plane of such a slot
};

// continuity-adjoint blocks over the nodes of a w x h-cell level (one
// partial-sum pair each)
size_t node_blocks(int w, int h) {
  return (size_t)((w + kAdjContTX) / kAdjContTX) * (size_t)((h + kAdjContTY) / kAdjContTY);
}

// The tape for `steps` base steps, a checkpoint every `every`, when every
// patch of the run spans at most frows fine node rows (<= 0 or more than
// the fine grid has: all of them).  The fine planes of the checkpoints and
// of the stored steps hold only those rows; the adjoint state spans the
// whole fine grid.
TapeLayout tape_layout(const dmr_params* p, int64_t steps, int every, int frows) {
  const Layout L = layout_of(p);
  const size_t f = sizeof(float);
  const int full = refined(p) ? p->r * p->ny + 1 : 0;
  TapeLayout T;
  T.frows = (frows <= 0 || frows > full) ? full : frows;
  T.fplane = (size_t)T.frows * (size_t)L.pitch1;
  size_t off = 0;
  T.adj_c = off; off += align256(L.plane0 * kAdjPlanes * f);
  T.adj_f = off; off += align256(L.plane1 * kAdjPlanes * f);
  T.nck = (int)((steps + every - 1) / every);
  T.ck_size = align256((L.plane0 * kCkC + T.fplane * kCkF) * f);
  T.ck = off; off += T.ck_size * (size_t)(T.nck + 1);
  T.ring0 = off; off += align256(L.plane0 * kRing * f);
  T.st_size = align256((L.plane0 * kStC + T.fplane * kStF) * f);
  // coarse steps per window block (as level_coeffs derives them)
  const int spb = (int)std::lround(p->cells_per_lambda / p->courant) / kRing;
  T.nbk = every / std::max(spb, 1) + 2;
  T.nlog = (int)(steps / std::max(spb, 1)) + 2;
  T.rlog = off; off += align256(L.plane0 * f) * (size_t)T.nlog;
  T.bk_size = align256((L.plane0 * kBkC + T.fplane * kBkF) * f);
  T.last_size = align256(T.fplane * 2 * f);
  T.bank_size = T.st_size * (size_t)every + T.bk_size * (size_t)T.nbk + T.last_size;
  T.store = off; off += T.bank_size * 2;  // two banks: replay / reverse overlap
  T.src_size = align256((size_t)2 * p->ny * f);
  T.src = off; off += T.src_size * (size_t)every;
  T.u = off; off += align256((size_t)2 * steps * sizeof(double));
  T.part_per_step = node_blocks(p->nx, p->ny) +
                    (refined(p) ? node_blocks(p->r * p->nx, p->r * p->ny) : 0);
  T.part = off; off += align256(T.part_per_step * 2 * sizeof(double) * (size_t)every);
  T.gsum = off; off += 256;
  T.wpart = off; off += align256(1024 * sizeof(double));
  T.total = off;
  return T;
}

struct AdjLevel {
  float* hz[2] = {nullptr, nullptr};
  float *ex = nullptr, *ey = nullptr, *jx = nullptr, *jy = nullptr, *n = nullptr,
        *acc = nullptr, *ring = nullptr;
  // second buffers of lam E, J: an EM adjoint launch reads one and writes
  // the other (flip() swaps them, with the two lam Hz buffers)
  float *ex2 = nullptr, *ey2 = nullptr, *jx2 = nullptr, *jy2 = nullptr;
  // patch: g of substeps 1 (gx, gy) and 2 (g2x, g2y) for Eq. (5b) transposed
  float *gx = nullptr, *gy = nullptr, *g2x = nullptr, *g2y = nullptr;
  float *n2 = nullptr, *hx = nullptr;  // n2: second lam n buffer (continuity)
  int cur = 0;
  void flip() {
    cur = 1 - cur;
    std::swap(ex, ex2); std::swap(ey, ey2); std::swap(jx, jx2); std::swap(jy, jy2);
  }
};

AdjLevel adj_carve(char* base, size_t plane) {
  AdjLevel a;
  float* q = (float*)base;
  auto take = [&](size_t k) { float* r = q; q += k * plane; return r; };
  a.hz[0] = take(1); a.hz[1] = take(1);
  a.ex = take(1); a.ey = take(1); a.jx = take(1); a.jy = take(1);
  a.n = take(1); a.acc = take(1); a.ring = take(kRing);
  a.gx = take(1); a.gy = take(1); a.ex2 = take(1); a.ey2 = take(1);
  a.jx2 = take(1); a.jy2 = take(1); a.n2 = take(1); a.hx = take(1);
  a.g2x = take(1); a.g2y = take(1);
  return a;
}

// stored values of step k (global index) of the segment starting at step
// k0, in a bank.  The fine planes hold fine rows [row0, row0 + T.frows)
// (row0: the first row of the segment's last patch, which contains every
// patch of the segment); the pointers handed out are offset so that entity
// (i, j) of the fine grid is at j * pitch + i, as the kernels address it
// (only the patch rows are ever accessed).  Steps of one window block share
// its density and E_rms^2 slot; every step of the segment shares the slot of
// the patch E after the last substep (stored and read for the last step only).
StepStore store_slot(const dmr_sim* s, const TapeLayout& T, int64_t k, int64_t k0, int bank,
                     int row0) {
  const int spb = std::max(s->L0.spb, 1);
  const int blk = (int)(k / spb - k0 / spb);
  char* bank0 = s->tape.base + T.store + T.bank_size * (size_t)bank;
  float* b = (float*)(bank0 + T.st_size * (size_t)(k - k0));
  float* bb = (float*)(bank0 + T.st_size * (size_t)s->tape.every + T.bk_size * (size_t)blk);
  float* bl = (float*)(bank0 + T.st_size * (size_t)s->tape.every + T.bk_size * (size_t)T.nbk);
  const size_t p0 = s->L0.plane, fp = T.fplane;
  const uintptr_t rowoff = (uintptr_t)row0 * s->L1.pitch * sizeof(float);
  StepStore ss;
  ss.cexi = b; ss.ceyi = b + p0; ss.cexp = b + 2 * p0; ss.ceyp = b + 3 * p0;
  ss.cn = bb; ss.ce2 = bb + p0;
  auto pl = [&](float* base, int q) {
    return (float*)((uintptr_t)base - rowoff + (uintptr_t)q * fp * sizeof(float));
  };
  float* fs = b + kStC * p0;
  ss.fex0 = pl(fs, 0); ss.fey0 = pl(fs, 1); ss.fex1 = pl(fs, 2); ss.fey1 = pl(fs, 3);
  float* fb = bb + kBkC * p0;
  ss.fn = pl(fb, 0); ss.fe2 = pl(fb, 1);
  ss.fex2 = pl(bl, 0); ss.fey2 = pl(bl, 1);
  return ss;
}

float* ck_base(const dmr_sim* s, const TapeLayout& T, int idx) {
  return (float*)(s->tape.base + T.ck + T.ck_size * (size_t)idx);
}

// live planes of a checkpoint, in slot order
void ck_planes(dmr_sim* s, float* live_c[9], float* live_f[15]) {
  Level &C = s->L0, &F = s->L1;
  const int c = s->ccur, nc = s->ncur;
  float* cs[9] = {C.hz[c], C.hz[1 - c], C.ex[c], C.ey[c], C.jx[c], C.jy[c], C.n[nc], C.acc,
                  C.ring};
  for (int q = 0; q < 9; q++) live_c[q] = cs[q];
  float* fs[7] = {F.hz[0], F.ex[0], F.ey[0], F.jx[0], F.jy[0], F.n[nc], F.acc};
  for (int q = 0; q < 7; q++) live_f[q] = fs[q];
  for (int k = 0; k < kRing; k++) live_f[7 + k] = F.ring ? F.ring + (size_t)k * F.plane : nullptr;
}

// copy the live planes to / from a checkpoint or saved state at b: the
// coarse planes whole; the patch planes over the patch's rows, plane q of
// the buffer at q * fplane floats from its fine part, its row 0 being fine
// row rowbase (a saved state: full planes, rowbase 0; a tape checkpoint:
// planes of the tape's rows, rowbase the patch's first row)
// ring: with the coarse window planes (the live state's layout), else
// without them (a tape checkpoint)
int ck_copy(dmr_sim* s, float* b, bool save, size_t fplane, int rowbase, bool ring = true) {
  float *lc[9], *lf[15];
  ck_planes(s, lc, lf);
  const size_t p0 = s->L0.plane;
  CopyJobs J{};
  for (int q = 0; q < (ring ? 9 : 8); q++) {
    const size_t n = q == 8 ? kRing * p0 : p0;
    if (save) job(&J, lc[q], b + q * p0, n);
    else job(&J, b + q * p0, lc[q], n);
  }
  if (s->has_patch) {
    const Level& F = s->L1;
    const int row = s->p.r * s->ext[1];
    const size_t off = (size_t)row * F.pitch;
    const size_t n = (size_t)(s->p.r * (s->ext[3] - s->ext[1]) + 1) * F.pitch;
    float* fb = b + (ring ? kLiveC : kCkC) * p0 + (size_t)(row - rowbase) * F.pitch;
    for (int q = 0; q < kCkF; q++) {
      if (save) job(&J, lf[q] + off, fb + q * fplane, n);
      else job(&J, fb + q * fplane, lf[q] + off, n);
    }
  }
  return run_copies(s, J);
}

// fine node rows of the current patch (0 without one)
int patch_rows(const dmr_sim* s) {
  return s->has_patch ? s->p.r * (s->ext[3] - s->ext[1]) + 1 : 0;
}

int ck_save(dmr_sim* s, const TapeLayout& T, int idx, Ckpt* k) {
  if (patch_rows(s) > T.frows)
    return fail(s, DMR_ENOMEM, "the patch spans %d fine rows, the tape was sized for %d "
                               "(dmr_adjoint_tape_bytes_rows)", patch_rows(s), T.frows);
  k->step = s->step; k->blocks = s->blocks; k->ccur = s->ccur; k->ncur = s->ncur;
  k->has = s->has_patch; k->ty1 = s->ty1;
  for (int q = 0; q < 4; q++) k->ext[q] = s->ext[q];
  return ck_copy(s, ck_base(s, T, idx), true, T.fplane, s->p.r * s->ext[1], false);
}

int ck_restore(dmr_sim* s, const TapeLayout& T, int idx, const Ckpt& k) {
  s->step = k.step; s->blocks = k.blocks; s->ccur = k.ccur; s->ncur = k.ncur;
  s->has_patch = k.has != 0; s->ty1 = k.ty1;
  for (int q = 0; q < 4; q++) s->ext[q] = k.ext[q];
  if (int rc = ck_copy(s, ck_base(s, T, idx), false, T.fplane, s->p.r * s->ext[1], false)) return rc;
  // coarse window plane q: the last block b < k.blocks with b = q (mod kRing)
  // closed during the recording (which starts at block 0), else the ring at
  // its start
  const size_t p0 = s->L0.plane, lsz = align256(p0 * sizeof(float));
  CopyJobs J{};
  for (int q = 0; q < kRing; q++) {
    const float* src = (const float*)(s->tape.base + T.ring0) + (size_t)q * p0;
    if (k.blocks - 1 >= q) {
      const int64_t b = q + (int64_t)kRing * ((k.blocks - 1 - q) / kRing);
      if (b >= T.nlog) return fail(s, DMR_EINVAL, "window block %lld beyond the tape's log", (long long)b);
      src = (const float*)(s->tape.base + T.rlog + lsz * (size_t)b);
    }
    job(&J, (float*)src, s->L0.ring + (size_t)q * p0, p0);
  }
  return run_copies(s, J);
}

AdjEMArgs adj_em_args(const dmr_sim* s, const Level& Lv, AdjLevel& a, bool fine,
                      const int reg[4]) {
  const dmr_params& p = s->p;
  AdjEMArgs A{};
  A.L = reg[0]; A.B = reg[1]; A.R = reg[2]; A.T = reg[3];
  A.pitch = Lv.pitch;
  A.S = Lv.S; A.c1 = Lv.c1; A.a = Lv.a; A.kn = Lv.kn; A.cmur = Lv.cmur;
  A.gamma = fine ? (float)p.fine_filter : 0.f;
  A.fine = fine ? 1 : 0;
  A.bc_x = p.bc_x; A.bc_y = p.bc_y;
  A.is = fine ? -1 : p.tfsf_i;
  A.lhz_in = a.hz[a.cur]; A.lhz_out = a.hz[1 - a.cur];
  A.lex = a.ex; A.ley = a.ey; A.ljx = a.jx; A.ljy = a.jy; A.lacc = a.acc;
  A.lex_o = a.ex2; A.ley_o = a.ey2; A.ljx_o = a.jx2; A.ljy_o = a.jy2;
  A.gx = a.gx; A.gy = a.gy;
  A.ln = a.n;
  return A;
}

AdjContArgs adj_cont_args(const dmr_sim* s, const Level& Lv, AdjLevel& a, bool fine,
                          const int reg[4]) {
  const dmr_params& p = s->p;
  AdjContArgs K{};
  K.L = reg[0]; K.B = reg[1]; K.R = reg[2]; K.T = reg[3];
  K.pitch = Lv.pitch; K.plane = Lv.plane; K.fine = fine ? 1 : 0;
  K.inv_spp = (float)(1.0 / Lv.spp);
  K.dtn = (float)(Lv.spb * Lv.dt);
  K.inv_dx2 = (float)(1.0 / (Lv.dx * Lv.dx));
  K.eeff_p2 = (float)(s->eeff / (1.0e4 * p.p_torr * p.p_torr));
  K.half_beta = (float)(0.5 * p.beta_ion);
  K.att = (float)std::pow(p.ecr_over_p, p.beta_ion);
  K.nuA = (float)(s->nu_m * p.A_ion);
  K.nu_m = (float)s->nu_m;
  K.ln_c = (float)std::log(p.ecr_over_p);
  K.inv_namb = (float)(1.0 / s->n_amb);
  K.De = (float)s->De; K.Da = (float)s->Da;
  K.d_const_mode = p.d_mode == DMR_D_CONST;
  K.d_const = (float)p.d_const;
  if (p.source_model == DMR_SOURCE_TOWNSEND) {  // the forward's constants
    const double mu_e = kQe / (kMe * s->nu_m);
    K.town = 1;
    K.tK = (float)(1.0e4 * p.A_town * p.p_torr * p.p_torr * mu_e);
    K.tB = (float)p.B_town;
    K.tatt = (float)p.nu_att;
  }
  K.rei = (float)rei_of(p);
  K.ln = a.n; K.ln_o = a.n2; K.lacc = a.acc; K.lring = a.ring;
  return K;
}

AdjGrowArgs adj_grow_args(const dmr_sim* s, AdjLevel& ac, AdjLevel& af, bool had,
                          const int old[4], const int neu[4], bool with_n) {
  const dmr_params& p = s->p;
  const int r = p.r;
  AdjGrowArgs G{};
  G.L = r * neu[0]; G.B = r * neu[1]; G.R = r * neu[2]; G.T = r * neu[3];
  if (had) { G.oL = r * old[0]; G.oB = r * old[1]; G.oR = r * old[2]; G.oT = r * old[3]; }
  G.cL = std::max(0, neu[0] - 1); G.cB = std::max(0, neu[1] - 1);
  G.cR = std::min(p.nx, neu[2] + 1); G.cT = std::min(p.ny, neu[3] + 1);
  G.cNX = p.nx; G.cNY = p.ny;
  G.pitch = s->L1.pitch; G.cpitch = s->L0.pitch;
  G.plane = s->L1.plane; G.cplane = s->L0.plane;
  G.with_n = with_n ? 1 : 0;
  G.lhz = af.hz[af.cur]; G.lex = af.ex; G.ley = af.ey; G.ljx = af.jx; G.ljy = af.jy;
  G.ln = af.n; G.lacc = af.acc; G.lring = af.ring;
  G.chz = ac.hz[ac.cur]; G.chz_prev = ac.hx; G.cex = ac.ex; G.cey = ac.ey;
  G.cjx = ac.jx; G.cjy = ac.jy; G.cn = ac.n; G.cacc = ac.acc; G.cring = ac.ring;
  return G;
}

// adjoint of base step k (meta: what the replay did; ss: its stored values)
int adj_step(dmr_sim* s, const TapeLayout& T, AdjLevel& ac, AdjLevel& af, int kk,
             const StepMeta& m, const StepStore& ss, const StepStore* nxt, size_t* npart) {
  const dmr_params& p = s->p;
  const Level &C = s->L0, &F = s->L1;
  const int r = p.r;
  const int creg[4] = {0, 0, p.nx, p.ny};
  const int freg[4] = {r * m.ext[0], r * m.ext[1], r * m.ext[2], r * m.ext[3]};
  double* part = (double*)(s->tape.base + T.part);
  hipError_t e = hipSuccess;
  if (m.grow) {  // Eq. (5a) prolongation after the step
    const AdjGrowArgs G = adj_grow_args(s, ac, af, m.has, m.ext, m.gnew, true);
    e = launch_adj_grow(G, s->st);
    if (e == hipSuccess)
      e = launch_adj_grow_clear(G, af.hz[af.cur], af.ex, af.ey, af.jx, af.jy, af.n, af.acc,
                                af.ring, s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint growth launch");
  }
  if (m.sync) {  // window close, continuity, density transfers
    AdjContArgs K = adj_cont_args(s, C, ac, false, creg);
    K.slot = m.slot; K.update = m.update;
    AdjContArgs G{};
    if (m.has) {
      G = adj_cont_args(s, F, af, true, freg);
      G.slot = m.slot; G.update = m.update;
    }
    if (m.update) {
      if (m.has) {
        AdjInjArgs I{m.ext[0], m.ext[1], m.ext[2], m.ext[3], F.pitch, C.pitch, ac.n, af.n};
        e = launch_adj_inj(I, s->st);
        if (e != hipSuccess) return hipfail(s, e, "adjoint transfer launch");
      }
      int np = 0;
      K.n = ss.cn; K.e2 = ss.ce2;
      if (m.has) { G.n = ss.fn; G.e2 = ss.fe2; }
      G.part = K.part = part + 2 * *npart;  // patch blocks first, then the base level
      e = launch_adj_cont(G, K, m.has ? 1 : 0, &np, s->st);
      *npart += (size_t)np;
      std::swap(ac.n, ac.n2);
      if (m.has) std::swap(af.n, af.n2);
    } else {
      e = launch_adj_close(K, s->st);
      if (e == hipSuccess && m.has) e = launch_adj_close(G, s->st);
    }
    if (e != hipSuccess) return hipfail(s, e, "adjoint continuity launch");
  }
  // patch substep m's adjoint arguments
  auto fine_args = [&](int sub) {
    AdjEMArgs A = adj_em_args(s, F, af, true, freg);
    A.exi = sub == 2 ? ss.fex1 : ss.fex0;
    A.eyi = sub == 2 ? ss.fey1 : ss.fey0;
    // E after substep 2 = the next step's stored E entering (the last
    // step of a segment stores it itself)
    A.exo = sub == 2 ? (nxt ? nxt->fex0 : ss.fex2) : ss.fex1;
    A.eyo = sub == 2 ? (nxt ? nxt->fey0 : ss.fey2) : ss.fey1;
    A.n = ss.fn;
    A.gx = sub == 2 ? af.g2x : af.gx;
    A.gy = sub == 2 ? af.g2y : af.gy;
    A.I0 = m.ext[0]; A.J0 = m.ext[1]; A.I1 = m.ext[2]; A.J1 = m.ext[3];
    A.cpitch = C.pitch;
    if (sub == 2) {  // the fine -> coarse transfer folded into substep 2
      A.rhz = ac.hz[ac.cur]; A.rex = ac.ex; A.rey = ac.ey; A.rjx = ac.jx; A.rjy = ac.jy;
    }
    return A;
  };
  if (m.has) {  // substep 2
    e = launch_adj_em(fine_args(2), s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint fine EM launch");
    af.flip();
  }
  AdjEMArgs A = adj_em_args(s, C, ac, false, creg);
  A.exi = ss.cexi; A.eyi = ss.ceyi; A.exo = ss.cexp; A.eyo = ss.ceyp; A.n = ss.cn;
  A.hz_extra = ac.hx;
  if (m.has) {  // Eq. (5b) transposed and the patch interior, folded in
    A.has_patch = 1;
    A.I0 = m.ext[0]; A.J0 = m.ext[1]; A.I1 = m.ext[2]; A.J1 = m.ext[3];
    A.fL = freg[0]; A.fB = freg[1]; A.fR = freg[2]; A.fT = freg[3];
    A.fpitch = F.pitch;
    A.g2x = af.g2x; A.g2y = af.g2y;
    // substep 1's boundary G from its inputs (lam leaving it: after the flip)
    A.s1ex = af.ex; A.s1ey = af.ey; A.s1jx = af.jx; A.s1jy = af.jy;
    A.s1exo = ss.fex1; A.s1eyo = ss.fey1; A.s1acc = af.acc; A.s1n = ss.fn;
    A.s1kn = F.kn;
  }
  if (p.tfsf_i > 0) {
    float* src = (float*)(s->tape.base + T.src + T.src_size * (size_t)kk);
    A.src_e = src;
    A.src_h = src + p.ny;
  }
  if (m.has) {  // substep 1 and the base level: one launch
    e = launch_adj_em_pair(fine_args(1), A, s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint EM launch");
    af.flip();
  } else {
    e = launch_adj_em(A, s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint base EM launch");
  }
  ac.flip();
  return DMR_OK;
}

// ---- state save / load (checkpoint and restart) -----------------------------
// Layout: a 256-byte header, then the planes of one checkpoint (16 base-level
// planes: Hz at n+1/2 and n-1/2, Ex, Ey, Jx, Jy, n, acc, 8 window slots; 15
// patch planes: Hz, Ex, Ey, Jx, Jy, n, acc, 8 slots, of which only the
// patch's rows are written).
struct StateHeader {
  char magic[8];
  uint32_t version, header_bytes;
  uint64_t params_hash, total_bytes;
  int64_t step, blocks;
  int32_t has_patch, ext[4], ty1;
};
static_assert(sizeof(StateHeader) <= 256, "header fits its slot");
constexpr size_t kStateHeader = 256;

uint64_t params_hash(const dmr_params& p) {
  // FNV-1a over the named fields (padding and the pad_ fields left out)
  const unsigned char* b = (const unsigned char*)&p;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](size_t lo, size_t hi) {
    for (size_t k = lo; k < hi; k++) h = (h ^ b[k]) * 1099511628211ull;
  };
  mix(0, offsetof(dmr_params, pad_));
  mix(offsetof(dmr_params, freq_hz), offsetof(dmr_params, pad2_));
  mix(offsetof(dmr_params, n_line), offsetof(dmr_params, pad3_));
  mix(offsetof(dmr_params, A_town), sizeof(dmr_params));
  return h;
}

// the live planes of a saved state (the patch planes over the whole fine
// grid); the union-of-blocks level appends its block map (one byte per block)
size_t state_planes_bytes(const dmr_params* p) {
  const Layout L = layout_of(p);
  const size_t fplane = (size_t)(refined(p) ? p->r * p->ny + 1 : 0) * (size_t)L.pitch1;
  return align256((L.plane0 * kLiveC + fplane * kCkF) * sizeof(float));
}
size_t state_bytes(const dmr_sim* s) {
  return kStateHeader + state_planes_bytes(&s->p) + (s->uni ? align256(s->h_act.size()) : 0);
}
size_t state_map_offset(const dmr_sim* s) { return kStateHeader + state_planes_bytes(&s->p); }

// host-side copy of the live planes to / from a host buffer b (floats after
// the header), the patch planes over the patch's rows only
int state_host_copy(dmr_sim* s, float* b, bool save) {
  float *lc[9], *lf[15];
  ck_planes(s, lc, lf);
  const size_t p0 = s->L0.plane, p1 = s->L1.plane;
  auto cp = [&](float* live, float* host, size_t n) {
    return save ? hipMemcpyAsync(host, live, n * 4, hipMemcpyDeviceToHost, s->st)
                : hipMemcpyAsync(live, host, n * 4, hipMemcpyHostToDevice, s->st);
  };
  for (int q = 0; q < 9; q++) {
    const hipError_t e = cp(lc[q], b + q * p0, q == 8 ? kRing * p0 : p0);
    if (e != hipSuccess) return hipfail(s, e, "state copy");
  }
  if (s->has_patch) {
    const size_t off = (size_t)(s->p.r * s->ext[1]) * s->L1.pitch;
    const size_t n = (size_t)(s->p.r * (s->ext[3] - s->ext[1]) + 1) * s->L1.pitch;
    float* fb = b + kLiveC * p0;
    for (int q = 0; q < kCkF; q++) {
      const hipError_t e = cp(lf[q] + off, fb + q * p1 + off, n);
      if (e != hipSuccess) return hipfail(s, e, "state copy");
    }
  }
  HIPCHK(s, hipStreamSynchronize(s->st));
  return DMR_OK;
}

}  // namespace

extern "C" {

int dmr_adjoint_tape_bytes(const dmr_params* p, int64_t steps, int ckpt_every, size_t* bytes) {
  return dmr_adjoint_tape_bytes_rows(p, steps, ckpt_every, 0, bytes);
}

int dmr_adjoint_tape_bytes_rows(const dmr_params* p, int64_t steps, int ckpt_every,
                                int32_t fine_rows, size_t* bytes) {
  std::string why;
  const int rc = check_params(p, &why);
  if (rc) return rc;
  if (!bytes || steps < 1 || ckpt_every < 1) return DMR_EINVAL;
  *bytes = tape_layout(p, steps, ckpt_every, fine_rows).total;
  return DMR_OK;
}

int dmr_forward_record(dmr_sim* s, int64_t steps, int ckpt_every, void* d_tape, size_t bytes) {
  if (!s) return DMR_EINVAL;
  if (steps < 1 || ckpt_every < 1) return fail(s, DMR_EINVAL, "steps and ckpt_every must be >= 1");
  if (s->step != 0) return fail(s, DMR_EINVAL, "recording starts at t = 0 (fresh handle)");
  if (refined(&s->p) && s->p.r != 2) return fail(s, DMR_EINVAL, "the adjoint supports r = 2");
  if (s->uni) return fail(s, DMR_EINVAL, "the adjoint supports the rectangular patch");
  if (!d_tape || ((uintptr_t)d_tape & 255)) return fail(s, DMR_EINVAL, "tape must be 256-byte aligned");
  // the most fine rows per slot the tape affords (its layout is linear in
  // them; the patch must never span more)
  const int full = refined(&s->p) ? s->p.r * s->p.ny + 1 : 0;
  int frows = full;
  if (tape_layout(&s->p, steps, ckpt_every, full).total > bytes) {
    int lo = 0, hi = full;  // lo fits (0 rows: no patch), hi does not
    if (tape_layout(&s->p, steps, ckpt_every, 1).total > bytes) hi = 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (tape_layout(&s->p, steps, ckpt_every, mid).total <= bytes) lo = mid;
      else hi = mid;
    }
    frows = lo;
  }
  if (frows < patch_rows(s) || (frows == 0 && refined(&s->p)))
    return fail(s, DMR_ENOMEM, "tape needs %zu bytes for the current patch (%d fine rows)",
                tape_layout(&s->p, steps, ckpt_every, std::max(patch_rows(s), 1)).total,
                patch_rows(s));
  const TapeLayout T = tape_layout(&s->p, steps, ckpt_every, frows);
  AdjTape& tp = s->tape;
  tp = AdjTape{};
  tp.base = (char*)d_tape;
  tp.bytes = bytes;
  tp.steps = steps;
  tp.every = ckpt_every;
  tp.nck = T.nck;
  tp.frows = T.frows;
  tp.ck.resize(T.nck);
  {  // the coarse window planes at the start
    CopyJobs J{};
    job(&J, s->L0.ring, (float*)(tp.base + T.ring0), kRing * s->L0.plane);
    if (int rc = run_copies(s, J)) return rc;
  }
  const size_t lsz = align256(s->L0.plane * sizeof(float));
  for (int64_t k = 0; k < steps; k++) {
    if (k % ckpt_every == 0) {
      const int idx = (int)(k / ckpt_every);
      if (int rc = ck_save(s, T, idx, &tp.ck[idx])) return rc;
    }
    StepCtx cx;
    if (int rc = base_step(s, &cx)) return rc;
    if (cx.meta.sync) {  // block blocks - 1 closed: log its coarse window plane
      const int64_t b = s->blocks - 1;
      if (b >= T.nlog) return fail(s, DMR_EINVAL, "window block %lld beyond the tape's log", (long long)b);
      CopyJobs J{};
      job(&J, s->L0.ring + (size_t)cx.meta.slot * s->L0.plane,
          (float*)(tp.base + T.rlog + lsz * (size_t)b), s->L0.plane);
      if (int rc = run_copies(s, J)) return rc;
    }
    if (cx.meta.grow) {
      Growth g;
      g.after = k + 1;
      for (int q = 0; q < 4; q++) g.ext[q] = cx.meta.gnew[q];
      tp.grow.push_back(g);
    }
  }
  if (int rc = ck_save(s, T, T.nck, &tp.fin)) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hipfail(s, e, "record");
  tp.valid = true;
  return DMR_OK;
}

int dmr_backward(dmr_sim* s, const void* d_tape, const float* d_w_coarse,
                 const float* d_w_fine, float* d_grad_seed, float* d_grad_seed_fine,
                 double grad[3]) {
  if (!s) return DMR_EINVAL;
  AdjTape& tp = s->tape;
  if (!tp.valid || d_tape != (const void*)tp.base)
    return fail(s, DMR_EINVAL, "no recorded run on this tape");
  if (!d_w_coarse) return fail(s, DMR_EINVAL, "coarse weights are required");
  const dmr_params& p = s->p;
  const TapeLayout T = tape_layout(&p, tp.steps, tp.every, tp.frows);
  const Level &C = s->L0, &F = s->L1;
  const int r = p.r;
  const bool ref = refined(&p);
  AdjLevel ac = adj_carve(tp.base + T.adj_c, C.plane);
  AdjLevel af = ref ? adj_carve(tp.base + T.adj_f, F.plane) : AdjLevel{};
  HIPCHK(s, hipMemsetAsync(tp.base + T.adj_c, 0, T.ck - T.adj_c, s->st));
  HIPCHK(s, hipMemsetAsync(tp.base + T.gsum, 0, 256, s->st));
  HIPCHK(s, hipMemsetAsync(tp.base + T.src, 0, T.src_size * (size_t)tp.every, s->st));
  // objective: lam n at t_final = the weights
  hipError_t e = launch_scatter(d_w_coarse, p.nx + 1, p.ny + 1, 1.f, ac.n, C.pitch, 0, 0, s->st);
  if (e == hipSuccess && ref && d_w_fine)
    e = launch_scatter(d_w_fine, r * p.nx + 1, r * p.ny + 1, 1.f, af.n, F.pitch, 0, 0, s->st);
  if (e != hipSuccess) return hipfail(s, e, "weights launch");
  // incident values per unit amplitude, E0 g sin(...) / E0 (Sec. II.B)
  {
    std::vector<double> u((size_t)2 * tp.steps, 0.0);
    if (p.tfsf_i > 0) {
      const double xs = p.tfsf_i * C.dx;
      for (int64_t k = 0; k < tp.steps; k++) {
        u[2 * k] = ey_inc(s, xs, (double)k * C.dt) / s->e0;
        u[2 * k + 1] = ey_inc(s, xs - 0.5 * C.dx, ((double)k + 0.5) * C.dt) / s->e0;
      }
    }
    HIPCHK(s, hipMemcpyAsync(tp.base + T.u, u.data(), u.size() * sizeof(double),
                             hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
  }
  // Reverse sweep, segments from the last: segment s is replayed on a
  // private stream into store bank s % 2 while the reverse kernels of
  // segment s + 1 run on the caller's stream from the other bank.
  hipStream_t user = s->st;
  if (!s->rep_st) {
    HIPCHK(s, hipStreamCreateWithFlags(&s->rep_st, hipStreamNonBlocking));
    for (int b = 0; b < 2; b++) {
      HIPCHK(s, hipEventCreateWithFlags(&s->ev_rep[b], hipEventDisableTiming));
      HIPCHK(s, hipEventCreateWithFlags(&s->ev_adj[b], hipEventDisableTiming));
    }
    HIPCHK(s, hipEventCreateWithFlags(&s->ev_sync, hipEventDisableTiming));
  }
  hipStream_t rep = s->rep_st;
  HIPCHK(s, hipEventRecord(s->ev_sync, user));
  HIPCHK(s, hipStreamWaitEvent(rep, s->ev_sync, 0));
  std::vector<StepMeta> meta((size_t)tp.every);
  for (int seg = tp.nck - 1; seg >= 0; seg--) {
    const int bank = seg & 1;
    const int64_t k0 = (int64_t)seg * tp.every;
    const int64_t k1 = std::min(tp.steps, k0 + tp.every);
    // replay into this bank once the reverse sweep that read it is done
    if (seg + 2 <= tp.nck - 1) HIPCHK(s, hipStreamWaitEvent(rep, s->ev_adj[bank], 0));
    s->st = rep;
    // the bank's fine rows start at the first row of the segment's last
    // patch (growth is monotone: it contains the segment's earlier patches)
    const Ckpt& ke = seg + 1 < tp.nck ? tp.ck[seg + 1] : tp.fin;
    const int row0 = ke.has ? r * ke.ext[1] : 0;
    int rc = ck_restore(s, T, seg, tp.ck[seg]);
    for (int64_t k = k0; k < k1 && !rc; k++) {
      StepCtx cx;
      cx.store = true;
      cx.last = k == k1 - 1;
      cx.ss = store_slot(s, T, k, k0, bank, row0);
      cx.forced = true;
      for (const Growth& g : tp.grow)
        if (g.after == k + 1) {
          cx.force_grow = true;
          for (int q = 0; q < 4; q++) cx.force_ext[q] = g.ext[q];
        }
      rc = base_step(s, &cx);
      meta[(size_t)(k - k0)] = cx.meta;
    }
    s->st = user;
    if (rc) return rc;
    HIPCHK(s, hipEventRecord(s->ev_rep[bank], rep));
    HIPCHK(s, hipStreamWaitEvent(user, s->ev_rep[bank], 0));
    size_t npart = 0;
    for (int64_t k = k1 - 1; k >= k0; k--) {
      const int kk = (int)(k - k0);
      const StepStore ss = store_slot(s, T, k, k0, bank, row0);
      const StepStore nx = store_slot(s, T, k + 1, k0, bank, row0);
      if (int rc2 = adj_step(s, T, ac, af, kk, meta[kk], ss, k == k1 - 1 ? nullptr : &nx, &npart))
        return rc2;
    }
    e = launch_adj_reduce((const float*)(tp.base + T.src), (int)(k1 - k0),
                          (int)(T.src_size / sizeof(float)), p.ny,
                          (const double*)(tp.base + T.u) + 2 * k0,
                          (const double*)(tp.base + T.part), (int)npart,
                          (double*)(tp.base + T.gsum), s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint reduction launch");
    HIPCHK(s, hipEventRecord(s->ev_adj[bank], user));
  }
  // the replay stream's work (the live state) precedes the final restore
  HIPCHK(s, hipEventRecord(s->ev_sync, rep));
  HIPCHK(s, hipStreamWaitEvent(user, s->ev_sync, 0));
  // t = 0: the patch seeded from the coarse density (Eq. (5a))
  if (ref && s->had0) {
    const AdjGrowArgs G = adj_grow_args(s, ac, af, false, s->ext0, s->ext0, !s->keep_n0);
    e = launch_adj_grow(G, s->st);
    if (e != hipSuccess) return hipfail(s, e, "adjoint seed launch");
  }
  if (d_grad_seed) {
    e = launch_gather(ac.n, C.pitch, 0, 0, p.nx + 1, p.ny + 1, 1.f, d_grad_seed, s->st);
    if (e != hipSuccess) return hipfail(s, e, "gradient read-out");
  }
  if (d_grad_seed_fine && ref) {
    const int fw = r * p.nx + 1, fh = r * p.ny + 1;
    HIPCHK(s, hipMemsetAsync(d_grad_seed_fine, 0, (size_t)fw * fh * sizeof(float), s->st));
    if (s->had0 && s->keep_n0) {
      const int* x = s->ext0;
      e = launch_copy2d(af.n, F.pitch, r * x[0], r * x[1], d_grad_seed_fine, fw, r * x[0],
                        r * x[1], r * (x[2] - x[0]) + 1, r * (x[3] - x[1]) + 1, s->st);
      if (e != hipSuccess) return hipfail(s, e, "gradient read-out");
    }
  }
  double g3[3] = {0, 0, 0};
  HIPCHK(s, hipMemcpyAsync(g3, tp.base + T.gsum, sizeof(g3), hipMemcpyDeviceToHost, s->st));
  // back to t_final
  if (int rc = ck_restore(s, T, T.nck, tp.fin)) return rc;
  HIPCHK(s, hipStreamSynchronize(s->st));
  if (grad) for (int q = 0; q < 3; q++) grad[q] = g3[q];
  return DMR_OK;
}

int dmr_state_bytes(const dmr_sim* s, size_t* bytes) {
  if (!s || !bytes) return DMR_EINVAL;
  *bytes = state_bytes(s);
  return DMR_OK;
}

int dmr_save(dmr_sim* s, void* dst, size_t bytes, int dst_on_device) {
  if (!s || !dst) return DMR_EINVAL;
  const size_t need = state_bytes(s);
  if (bytes < need) return fail(s, DMR_ENOMEM, "state needs %zu bytes", need);
  if (dst_on_device && ((uintptr_t)dst & 255))
    return fail(s, DMR_EINVAL, "device state buffer must be 256-byte aligned");
  StateHeader h{};
  memcpy(h.magic, "DMRSTATE", 8);
  h.version = 1; h.header_bytes = (uint32_t)kStateHeader;
  h.params_hash = params_hash(s->p); h.total_bytes = need;
  h.step = s->step; h.blocks = s->blocks; h.has_patch = s->has_patch ? 1 : 0;
  for (int q = 0; q < 4; q++) h.ext[q] = s->ext[q];
  h.ty1 = s->ty1;
  float* body = (float*)((char*)dst + kStateHeader);
  char* map = (char*)dst + state_map_offset(s);
  if (dst_on_device) {
    if (int rc = ck_copy(s, body, true, s->L1.plane, 0)) return rc;
    HIPCHK(s, hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, s->st));
    if (s->uni)
      HIPCHK(s, hipMemcpyAsync(map, s->h_act.data(), s->h_act.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
  } else {
    if (int rc = state_host_copy(s, body, true)) return rc;
    memcpy(dst, &h, sizeof(h));
    if (s->uni) memcpy(map, s->h_act.data(), s->h_act.size());
  }
  return DMR_OK;
}

int dmr_load(dmr_sim* s, const void* src, size_t bytes, int src_on_device) {
  if (!s || !src) return DMR_EINVAL;
  const dmr_params& p = s->p;
  const size_t need = state_bytes(s);
  if (bytes < need) return fail(s, DMR_ENOMEM, "state needs %zu bytes", need);
  if (src_on_device && ((uintptr_t)src & 255))
    return fail(s, DMR_EINVAL, "device state buffer must be 256-byte aligned");
  StateHeader h{};
  const char* map = (const char*)src + state_map_offset(s);
  std::vector<uint8_t> act;
  if (s->uni) act.resize(s->h_act.size());
  if (src_on_device) {
    HIPCHK(s, hipStreamSynchronize(s->st));
    HIPCHK(s, hipMemcpy(&h, src, sizeof(h), hipMemcpyDeviceToHost));
    if (s->uni) HIPCHK(s, hipMemcpy(act.data(), map, act.size(), hipMemcpyDeviceToHost));
  } else {
    memcpy(&h, src, sizeof(h));
    if (s->uni) memcpy(act.data(), map, act.size());
  }
  if (memcmp(h.magic, "DMRSTATE", 8) != 0 || h.version != 1 || h.header_bytes != kStateHeader)
    return fail(s, DMR_EINVAL, "not a saved state");
  if (h.params_hash != params_hash(p) || h.total_bytes != need)
    return fail(s, DMR_EINVAL, "saved state belongs to other parameters");
  // every field of the header is checked before the handle changes: the
  // extents decide which fine rows the copy below writes
  if (h.step < 0 || h.blocks < 0 || (h.has_patch != 0 && h.has_patch != 1) ||
      (h.ty1 != 4 && h.ty1 != 8 && h.ty1 != 16))
    return fail(s, DMR_EINVAL, "saved state header out of range");
  if (h.has_patch && !refined(&p)) return fail(s, DMR_EINVAL, "saved state has a patch");
  if (h.has_patch) {
    const int* e = h.ext;
    const int Bk = p.block;
    const int xmin = p.mode == DMR_STATIC ? std::max(1, p.tfsf_i + 1) : block_xmin(p) * Bk;
    if (e[0] < xmin || e[1] < 1 || e[2] > p.nx - 1 || e[3] > p.ny - 1 || e[0] >= e[2] ||
        e[1] >= e[3])
      return fail(s, DMR_EINVAL, "saved patch extents outside the allowed region");
    if (p.mode == DMR_STATIC && !s->uni && memcmp(e, p.static_ext, sizeof(h.ext)) != 0)
      return fail(s, DMR_EINVAL, "saved patch differs from static_ext");
    if ((s->uni || p.regrid_rule == DMR_RULE_BLOCKS) && p.mode == DMR_DYNAMIC &&
        (e[0] % Bk || e[1] % Bk || e[2] % Bk || e[3] % Bk))
      return fail(s, DMR_EINVAL, "saved patch extents are not on the block grid");
  }
  if (s->uni) {
    // the block map: active blocks inside the margins, bounding box = extents
    const int NBx = p.nx / p.block, NBy = p.ny / p.block, xmin = block_xmin(p);
    int bb[4] = {NBx, NBy, 0, 0};
    for (int b = 0; b < NBx * NBy; b++) {
      if (act[b] > 1) return fail(s, DMR_EINVAL, "saved block map entry %d not 0/1", b);
      if (!act[b]) continue;
      const int bx = b % NBx, by = b / NBx;
      if (bx < xmin || by < 1 || bx > NBx - 2 || by > NBy - 2)
        return fail(s, DMR_EINVAL, "saved block %d outside the margins", b);
      bb[0] = std::min(bb[0], bx); bb[1] = std::min(bb[1], by);
      bb[2] = std::max(bb[2], bx + 1); bb[3] = std::max(bb[3], by + 1);
    }
    const bool any = bb[2] > bb[0];
    if (any != (h.has_patch != 0) ||
        (any && (bb[0] * p.block != h.ext[0] || bb[1] * p.block != h.ext[1] ||
                 bb[2] * p.block != h.ext[2] || bb[3] * p.block != h.ext[3])))
      return fail(s, DMR_EINVAL, "saved block map does not match the saved extents");
  }
  s->step = h.step; s->blocks = h.blocks; s->has_patch = h.has_patch != 0;
  for (int q = 0; q < 4; q++) s->ext[q] = h.ext[q];
  s->ty1 = h.ty1;
  s->tape.valid = false;  // a recorded run no longer describes this state
  float* body = (float*)((char*)src + kStateHeader);
  if (src_on_device) {
    if (int rc = ck_copy(s, body, false, s->L1.plane, 0)) return rc;
    HIPCHK(s, hipStreamSynchronize(s->st));
  } else {
    if (int rc = state_host_copy(s, body, false)) return rc;
  }
  if (!s->uni) return DMR_OK;
  memcpy(s->h_act.data(), act.data(), act.size());
  return union_install(s);
}

int dmr_weighted_sum(dmr_sim* s, int level, const float* d_w, double* out) {
  if (!s || !d_w || !out) return DMR_EINVAL;
  if (level != 0 && !(level == 1 && refined(&s->p)))
    return fail(s, DMR_EINVAL, "level %d not present", level);
  const Level& L = level == 0 ? s->L0 : s->L1;
  double* part = (double*)s->stage;  // 1024 partials + the result
  if (s->lay.off_stage + 1025 * sizeof(double) > s->lay.total)
    return fail(s, DMR_ENOMEM, "staging area too small");
  hipError_t e = launch_wdot(d_w, L.n[s->ncur], L.pitch, 0, 0, L.NX + 1, L.NY + 1, part,
                             part + 1024, s->st);
  if (e != hipSuccess) return hipfail(s, e, "weighted sum launch");
  HIPCHK(s, hipMemcpyAsync(out, part + 1024, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  return DMR_OK;
}

int dmr_weighted_sum_static(dmr_sim* s, int level, const float* d_w, double* out) {
  if (!s || !d_w || !out) return DMR_EINVAL;
  if (level != 0 && !(level == 1 && refined(&s->p)))
    return fail(s, DMR_EINVAL, "level %d not present", level);
  const Level& L = level == 0 ? s->L0 : s->L1;
  double* part = static_scratch(s->dev);
  if (!part)
    return fail(s, DMR_EHIP, "no address of the static scratch array on device %d", s->dev);
  // the same partial count as dmr_weighted_sum (so the same bits); the array
  // holds kStaticParts partials and the result
  const size_t n = (size_t)(L.NX + 1) * (L.NY + 1);
  const size_t nb = std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 1024));
  if (nb > (size_t)kStaticParts)
    return fail(s, DMR_EINVAL, "%zu partial sums exceed the static scratch array (%d)", nb,
                kStaticParts);
  hipError_t e = launch_wdot(d_w, L.n[s->ncur], L.pitch, 0, 0, L.NX + 1, L.NY + 1, part,
                             part + kStaticParts, s->st);
  if (e != hipSuccess) return hipfail(s, e, "weighted sum launch");
  HIPCHK(s, hipMemcpyAsync(out, part + kStaticParts, sizeof(double), hipMemcpyDeviceToHost,
                           s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  return DMR_OK;
}


}  // extern "C"

// ===========================================================================
// Batched form: many independent simulations advanced in lockstep.  Every
// per-step launch (base EM, two fine substeps, continuity on both levels)
// covers all instances through a block table; the steps of a steady regrid
// interval are captured once in a HIP graph and replayed.  Growth tests run
// per instance between intervals.
// ===========================================================================
struct dmr_batch {
  std::vector<dmr_sim*> sims;
  int count = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  char* ws = nullptr;
  std::string err;
  EMArgs* d_em = nullptr;      // [4 parities][count]
  EMArgs* d_fem = nullptr;     // [rf substeps][4 parities][count]
  int rf = 2;                  // fine substeps per coarse step (the refined instances' r)
  ContArgs* d_cont = nullptr;  // [2 density parities][count]
  ContArgs* d_fcont = nullptr; // [2][count]
  int2 *d_blk_base = nullptr, *d_blk_fine = nullptr, *d_blk_cont = nullptr,
       *d_blk_fcont = nullptr;
  int nblk_base = 0, nblk_fine = 0, nblk_cont = 0, nblk_fcont = 0;
  size_t cap_base = 0, cap_fine = 0, cap_cont = 0, cap_fcont = 0;  // table entries
  float2* d_src = nullptr;
  float2* h_src = nullptr;
  int64_t src_base = -1;
  int seg = 8, depth = 4, ty = 8;
  // subcycle schedule of the refined instances (all rectangles):
  // kSchedSeparate: base launch + one launch per fine substep;
  // kSchedFused: base launch + one two-substep patch launch (r = 4: two);
  // kSchedCombined: base step and both substeps in one launch (r = 2)
  int sched = 0;
  bool can_fuse = false, can_combine = false;
  EMArgs* d_fem2 = nullptr;   // two-substep patch args [pairs][4 parities][count]
  EMArgs* d_cem = nullptr;    // combined: base args, patch entities skipped [4][count]
  EMArgs* d_floc = nullptr;   // combined: patch args, boundary E local [4][count]
  int2* d_blk_comb = nullptr;
  int nblk_comb = 0;
  size_t cap_comb = 0;
  std::vector<EMArgs> h_fem2, h_cem, h_floc;
  std::vector<int2> h_blk_comb;
  bool use_graph = true, tuned = false, forced = false;
  hipGraphExec_t gexec = nullptr;
  bool graph_ok = false;
  // host copies of the tables (kept alive until their upload completes)
  std::vector<EMArgs> h_em, h_fem;
  std::vector<ContArgs> h_cont, h_fcont;
  std::vector<int2> h_blk_base, h_blk_fine, h_blk_cont, h_blk_fcont;
};

namespace {

constexpr int kSegCand[] = {2, 4, 8, 16, 32, 64};
constexpr int kTyCand[] = {4, 8, 16};
enum { kSchedSeparate = 0, kSchedFused = 1, kSchedCombined = 2 };

struct BatchLayout {
  std::vector<size_t> off, size;
  int rf = 2;  // r of the refined instances (all equal)
  size_t off_em = 0, off_fem = 0, off_cont = 0, off_fcont = 0, off_blk_base = 0,
         off_blk_fine = 0, off_blk_cont = 0, off_blk_fcont = 0, off_src = 0, total = 0;
  size_t off_fem2 = 0, off_cem = 0, off_floc = 0, off_blk_comb = 0;
  size_t cap_base = 0, cap_fine = 0, cap_cont = 0, cap_fcont = 0, cap_comb = 0;
};

int batch_layout(const dmr_params* p, int count, BatchLayout* L, std::string* why) {
  if (!p || count < 1) { *why = "count must be >= 1"; return DMR_EINVAL; }
  size_t off = 0;
  for (int k = count - 1; k >= 0; k--)
    if (refined(&p[k])) L->rf = p[k].r;
  for (int k = 0; k < count; k++) {
    int rc = check_params(&p[k], why);
    if (rc) return rc;
    if (refined(&p[k]) && p[k].r != L->rf) {
      *why = "refined instances of a batch must share r";
      return DMR_EINVAL;
    }
    if (refined(&p[k]) && p[k].r != 2 && p[k].regrid_rule == DMR_RULE_UNION) {
      *why = "the union-of-blocks level is r = 2";
      return DMR_EINVAL;
    }
    if (refined(&p[k]) && (p[k].regrid_rule == DMR_RULE_UNION) != (p[0].regrid_rule == DMR_RULE_UNION)) {
      *why = "instances must all or none use the union-of-blocks fine level";
      return DMR_EINVAL;
    }
    const double spp0 = p[0].cells_per_lambda / p[0].courant;
    const double sppk = p[k].cells_per_lambda / p[k].courant;
    if (std::fabs(spp0 - sppk) > 1e-9 || p[k].mode != p[0].mode ||
        p[k].continuity_on != p[0].continuity_on ||
        (p[k].mode == DMR_DYNAMIC && p[k].regrid_every != p[0].regrid_every)) {
      *why = "instances must share steps per period, mode, continuity and regrid cadence";
      return DMR_EINVAL;
    }
    const size_t b = layout_of(&p[k]).total;
    L->off.push_back(off);
    L->size.push_back(b);
    off += align256(b);
    const int nx = p[k].nx, ny = p[k].ny, r = refined(&p[k]) ? p[k].r : 1;
    // the shortest segment a batch may use (2 rows) gives the most blocks
    L->cap_base += (size_t)stream_blocks_x(nx) * stream_segments(ny, 2);
    L->cap_cont += (size_t)((nx + 1 + kTX - 1) / kTX) * ((ny + 1 + 3) / 4);
    if (refined(&p[k])) {
      const size_t t = (size_t)((r * nx + 1 + kTX - 1) / kTX) * ((r * ny + 1 + 3) / 4);
      L->cap_fine += t;
      L->cap_fcont += t;
    }
  }
  L->off_em = off;    off += align256(sizeof(EMArgs) * 4 * count);
  L->off_fem = off;   off += align256(sizeof(EMArgs) * 4 * L->rf * count);
  L->off_cont = off;  off += align256(sizeof(ContArgs) * 2 * count);
  L->off_fcont = off; off += align256(sizeof(ContArgs) * 2 * count);
  L->off_blk_base = off;  off += align256(sizeof(int2) * std::max<size_t>(L->cap_base, 1));
  L->off_blk_fine = off;  off += align256(sizeof(int2) * std::max<size_t>(L->cap_fine, 1));
  L->off_blk_cont = off;  off += align256(sizeof(int2) * std::max<size_t>(L->cap_cont, 1));
  L->off_blk_fcont = off; off += align256(sizeof(int2) * std::max<size_t>(L->cap_fcont, 1));
  L->off_src = off;       off += align256(sizeof(float2) * kSrcSteps * count);
  // the two-substep and combined schedules: their argument tables, and the
  // combined table (groups of 16 base waves <= 4-wave blocks, plus the tiles)
  L->off_fem2 = off;      off += align256(sizeof(EMArgs) * 4 * 2 * count);
  L->off_cem = off;       off += align256(sizeof(EMArgs) * 4 * count);
  L->off_floc = off;      off += align256(sizeof(EMArgs) * 4 * count);
  L->cap_comb = L->cap_base + L->cap_fine;
  L->off_blk_comb = off;  off += align256(sizeof(int2) * std::max<size_t>(L->cap_comb, 1));
  L->total = off;
  return DMR_OK;
}

int bfail(dmr_batch* b, int code, const char* what) {
  if (b) b->err = what;
  return code;
}

// rebuild block tables and argument arrays for the current configuration,
// parities and patches; uploads on the batch stream and waits
int batch_tables(dmr_batch* b) {
  const int n = b->count;
  b->h_em.assign(4 * n, EMArgs{});
  b->h_fem.assign(4 * b->rf * n, EMArgs{});
  b->h_cont.assign(2 * n, ContArgs{});
  b->h_fcont.assign(2 * n, ContArgs{});
  b->h_fem2.assign(4 * 2 * n, EMArgs{});
  b->h_cem.assign(4 * n, EMArgs{});
  b->h_floc.assign(4 * n, EMArgs{});
  b->h_blk_base.clear(); b->h_blk_fine.clear();
  b->h_blk_cont.clear(); b->h_blk_fcont.clear(); b->h_blk_comb.clear();
  // the two-substep and combined schedules need rectangular patches
  bool any_patch = false, any_union = false;
  for (const dmr_sim* s : b->sims) {
    any_patch = any_patch || s->has_patch;
    any_union = any_union || s->uni;
  }
  b->can_fuse = any_patch && !any_union;
  b->can_combine = b->can_fuse && b->rf == 2;
  if ((b->sched == kSchedFused && !b->can_fuse) || (b->sched == kSchedCombined && !b->can_combine))
    b->sched = kSchedSeparate;
  for (int k = 0; k < n; k++) {
    dmr_sim* s = b->sims[k];
    s->seg0 = b->seg;
    s->depth0 = b->depth;
    s->ty1 = b->ty;
    if (s->uni && (s->tyu != b->ty || !s->tyu_env)) {  // the batch's tile rows
      s->tyu = b->ty;
      s->tyu_env = true;
      if (int rc = union_install(s)) return bfail(b, rc, s->err.c_str());
    }
    for (int v = 0; v < 4; v++) {
      const int c = v & 1, nc = v >> 1;
      make_base_em(s, c, nc, &b->h_em[v * n + k]);
      if (s->has_patch)
        for (int m = 1; m <= b->rf; m++)
          make_fine_em(s, m, c, nc, b->ty, &b->h_fem[((m - 1) * 4 + v) * n + k]);
      b->h_cem[v * n + k] = b->h_em[v * n + k];
      if (!s->has_patch || s->uni) continue;
      // two-substep / combined launches read the patch state from one buffer
      // and write the other; the buffers swap every step (batch_advance), so
      // at coarse parity c the state is in buffer c ^ ccur of this build
      const Level &C = s->L0, &F = s->L1;
      const int rel = c ^ s->ccur;
      if (b->rf == 4) {  // substeps (1, 2) then (3, 4): buffer 0 -> 1 -> 0
        for (int h = 0; h < 2; h++) {
          EMArgs& G = b->h_fem2[(h * 4 + v) * n + k];
          make_fine_em(s, 2 * h + 2, c, nc, b->ty, &G);
          em_args_level(&G, F, h, 1 - h, F.n[nc], F.acc);
          G.frac = (float)(2 * h + 1) / 4.f;
          G.hz_save = nullptr;
          G.hz_lo = nullptr;
        }
      } else {
        EMArgs& G = b->h_fem2[v * n + k];
        make_fine_em(s, 2, c, nc, b->ty, &G);  // restriction targets
        em_args_level(&G, F, rel, 1 - rel, F.n[nc], F.acc);
        G.frac = 0.5f;  // time fraction of substep 1
        EMArgs& A = b->h_cem[v * n + k];
        A.skip_on = 1;
        A.sL = s->ext[0]; A.sB = s->ext[1]; A.sR = s->ext[2]; A.sT = s->ext[3];
        EMArgs& H = b->h_floc[v * n + k];
        H = G;
        H.chz0 = C.hz[c]; H.cjx0 = C.jx[c]; H.cjy0 = C.jy[c]; H.cn0 = C.n[nc];
        H.cS = C.S; H.cc1 = C.c1; H.ckn = C.kn; H.cis = s->p.tfsf_i;
        H.cnx = s->p.nx; H.cny = s->p.ny;
      }
    }
    for (int nc = 0; nc < 2; nc++) {
      make_base_cont(s, nc, &b->h_cont[nc * n + k]);
      if (s->has_patch) make_fine_cont(s, nc, &b->h_fcont[nc * n + k]);
    }
    const EMArgs& A = b->h_em[k];
    for (int t = 0; t < A.nbx * A.nseg; t++) b->h_blk_base.push_back(make_int2(k, t));
    const ContArgs& K = b->h_cont[k];
    const int cny = (K.T - K.B + 1 + 3) / 4;
    for (int t = 0; t < K.nbx * cny; t++) b->h_blk_cont.push_back(make_int2(k, t));
    if (s->has_patch && s->uni) {  // the instance's tile list
      for (int t = 0; t < s->ntiles; t++) {
        b->h_blk_fine.push_back(make_int2(k, t));
        b->h_blk_fcont.push_back(make_int2(k, t));
      }
    } else if (s->has_patch) {
      const EMArgs& G = b->h_fem[k];
      const int fny = (G.T - G.B + 1 + b->ty - 1) / b->ty;
      for (int t = 0; t < G.nbx * fny; t++) b->h_blk_fine.push_back(make_int2(k, t));
      const ContArgs& H = b->h_fcont[k];
      const int hny = (H.T - H.B + 1 + 3) / 4;
      for (int t = 0; t < H.nbx * hny; t++) b->h_blk_fcont.push_back(make_int2(k, t));
    }
  }
  // combined table: every instance's groups of 16 base waves, then the
  // patch tiles (the same 64 x ty tiles as h_blk_fine, coded -1 - t)
  for (int k = 0; k < n && b->can_combine; k++) {
    const EMArgs& A = b->h_em[k];
    const int groups = (A.nbx * (kThreads / 64) * A.nseg + kFineThreads / 64 - 1) / (kFineThreads / 64);
    for (int g = 0; g < groups; g++) b->h_blk_comb.push_back(make_int2(k, g));
  }
  if (b->can_combine)
    for (const int2& t : b->h_blk_fine) b->h_blk_comb.push_back(make_int2(t.x, -1 - t.y));
  if (b->h_blk_base.size() > b->cap_base || b->h_blk_fine.size() > b->cap_fine ||
      b->h_blk_cont.size() > b->cap_cont || b->h_blk_fcont.size() > b->cap_fcont ||
      b->h_blk_comb.size() > b->cap_comb)
    return bfail(b, DMR_EINVAL, "batch block table exceeds its workspace capacity");
  b->nblk_comb = (int)b->h_blk_comb.size();
  b->nblk_base = (int)b->h_blk_base.size();
  b->nblk_fine = (int)b->h_blk_fine.size();
  b->nblk_cont = (int)b->h_blk_cont.size();
  b->nblk_fcont = (int)b->h_blk_fcont.size();
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->st) : hipSuccess;
  };
  if (up(b->d_em, b->h_em.data(), b->h_em.size() * sizeof(EMArgs)) ||
      up(b->d_fem, b->h_fem.data(), b->h_fem.size() * sizeof(EMArgs)) ||
      up(b->d_cont, b->h_cont.data(), b->h_cont.size() * sizeof(ContArgs)) ||
      up(b->d_fcont, b->h_fcont.data(), b->h_fcont.size() * sizeof(ContArgs)) ||
      up(b->d_blk_base, b->h_blk_base.data(), b->h_blk_base.size() * sizeof(int2)) ||
      up(b->d_blk_fine, b->h_blk_fine.data(), b->h_blk_fine.size() * sizeof(int2)) ||
      up(b->d_blk_cont, b->h_blk_cont.data(), b->h_blk_cont.size() * sizeof(int2)) ||
      up(b->d_blk_fcont, b->h_blk_fcont.data(), b->h_blk_fcont.size() * sizeof(int2)) ||
      up(b->d_fem2, b->h_fem2.data(), b->h_fem2.size() * sizeof(EMArgs)) ||
      up(b->d_cem, b->h_cem.data(), b->h_cem.size() * sizeof(EMArgs)) ||
      up(b->d_floc, b->h_floc.data(), b->h_floc.size() * sizeof(EMArgs)) ||
      up(b->d_blk_comb, b->h_blk_comb.data(), b->h_blk_comb.size() * sizeof(int2)) ||
      hipStreamSynchronize(b->st))
    return bfail(b, DMR_EHIP, "batch table upload failed");
  b->graph_ok = false;
  return DMR_OK;
}

// incident values of steps [base, base + kSrcSteps) for every instance
int batch_sources(dmr_batch* b, int64_t base) {
  if (hipStreamSynchronize(b->st) != hipSuccess) return bfail(b, DMR_EHIP, "sync");
  for (int k = 0; k < b->count; k++)
    for (int q = 0; q < kSrcSteps; q++) {
      float ey, hz;
      incident_values(b->sims[k], base + q, &ey, &hz);
      b->h_src[(size_t)k * kSrcSteps + q] = make_float2(ey, hz);
    }
  if (hipMemcpyAsync(b->d_src, b->h_src, sizeof(float2) * kSrcSteps * b->count,
                     hipMemcpyHostToDevice, b->st) != hipSuccess)
    return bfail(b, DMR_EHIP, "source upload failed");
  b->src_base = base;
  return DMR_OK;
}

// host bookkeeping of one base step (parities, counters), shared by the
// eager and the graph paths; returns the continuity slot/update of the step
void batch_advance(dmr_batch* b, int* slot, int* update) {
  *slot = -1;
  *update = 0;
  const bool swap_fine = b->sched != kSchedSeparate && b->rf == 2;
  for (dmr_sim* s : b->sims) {
    if (swap_fine && s->has_patch) {  // the new patch state is in buffer 1
      Level& F = s->L1;
      std::swap(F.hz[0], F.hz[1]);
      std::swap(F.ex[0], F.ex[1]);
      std::swap(F.ey[0], F.ey[1]);
      std::swap(F.jx[0], F.jx[1]);
      std::swap(F.jy[0], F.jy[1]);
    }
    s->ccur = 1 - s->ccur;
    s->step++;
    if (s->p.continuity_on && s->step % s->L0.spb == 0) {
      *slot = (int)(s->blocks % kRing);
      s->blocks++;
      *update = s->blocks >= kRing;
      if (*update) s->ncur = 1 - s->ncur;
    }
  }
}

// queue one base step of every instance (no growth test)
int batch_launch_step(dmr_batch* b, hipEvent_t* tb, hipEvent_t* tf) {
  const int n = b->count;
  dmr_sim* s0 = b->sims[0];
  const int v = s0->ccur + 2 * s0->ncur;
  const int nc = s0->ncur;
  const int k = (int)(s0->step - b->src_base);
  const bool uni = s0->uni;
  if (tb) (void)hipEventRecord(tb[0], b->st);
  hipError_t e = hipSuccess;
  if (b->sched == kSchedCombined) {
    e = launch_dmr_step_batch(b->d_cem + v * n, b->d_floc + v * n, b->d_blk_comb, b->nblk_comb,
                              b->d_src, k, b->depth, b->ty, b->st);
    if (tb) (void)hipEventRecord(tb[1], b->st);
    if (tf) (void)hipEventRecord(tf[0], b->st);
    if (tf) (void)hipEventRecord(tf[1], b->st);
    if (e != hipSuccess) return bfail(b, DMR_EHIP, "batched combined step launch");
  } else {
    e = launch_em_stream_batch(b->d_em + v * n, b->d_blk_base, b->nblk_base, b->d_src, k,
                               b->depth, b->st);
    if (tb) (void)hipEventRecord(tb[1], b->st);
    if (e != hipSuccess) return bfail(b, DMR_EHIP, "batched base EM launch");
    if (tf) (void)hipEventRecord(tf[0], b->st);
    if (b->sched == kSchedFused) {
      for (int h = 0; h < (b->rf == 4 ? 2 : 1) && b->nblk_fine; h++) {
        e = launch_fine2_batch(b->d_fem2 + (h * 4 + v) * n, b->d_blk_fine, b->nblk_fine, b->ty,
                               b->rf == 4, b->st);
        if (e != hipSuccess) return bfail(b, DMR_EHIP, "batched two-substep launch");
      }
    } else {
      for (int m = 1; m <= b->rf && b->nblk_fine; m++) {
        const EMArgs* fa = b->d_fem + ((m - 1) * 4 + v) * n;
        e = uni ? launch_em_union_batch(fa, b->d_blk_fine, b->nblk_fine, b->ty, b->st)
                : launch_em_batch(fa, b->d_blk_fine, b->nblk_fine, b->ty, b->st);
        if (e != hipSuccess) return bfail(b, DMR_EHIP, "batched fine EM launch");
      }
    }
    if (tf) (void)hipEventRecord(tf[1], b->st);
  }
  int slot, update;
  batch_advance(b, &slot, &update);
  if (slot >= 0) {
    e = launch_cont_batch(b->d_cont + nc * n, b->d_blk_cont, b->nblk_cont, false, slot,
                          update, b->st);
    if (e == hipSuccess && uni)
      e = launch_cont_union_batch(b->d_fcont + nc * n, b->d_blk_fcont, b->nblk_fcont, b->ty,
                                  slot, update, b->st);
    else if (e == hipSuccess)
      e = launch_cont_batch(b->d_fcont + nc * n, b->d_blk_fcont, b->nblk_fcont, true, slot,
                            update, b->st);
    if (e != hipSuccess) return bfail(b, DMR_EHIP, "batched continuity launch");
  }
  return DMR_OK;
}

int batch_regrid(dmr_batch* b) {
  bool changed = false;
  for (dmr_sim* s : b->sims) {
    int old[4] = {s->ext[0], s->ext[1], s->ext[2], s->ext[3]};
    const bool had = s->has_patch;
    const int64_t gen = s->ugen;
    const int rc = regrid(s, false);
    if (rc) return bfail(b, rc, s->err.c_str());
    if (s->has_patch != had || memcmp(old, s->ext, sizeof(old)) || s->ugen != gen) changed = true;
  }
  return changed ? batch_tables(b) : DMR_OK;
}

// pick the streaming segment/depth and the fine tile height by timing real
// steps (all candidates give bit-identical results)
std::vector<std::pair<std::string, std::array<int, 4>>>& tune_cache() {
  static std::vector<std::pair<std::string, std::array<int, 4>>> c;
  return c;
}

std::string batch_key(const dmr_batch* b) {
  std::string k;
  for (const dmr_sim* s : b->sims) {
    char buf[64];
    snprintf(buf, sizeof(buf), "%dx%d:%d,%d,%d,%d;", s->p.nx, s->p.ny, s->ext[0], s->ext[1],
             s->ext[2], s->ext[3]);
    k += buf;
  }
  return k;
}

int batch_tune(dmr_batch* b, int64_t* used) {
  *used = 0;
  const std::string key = batch_key(b);
  for (auto& kv : tune_cache())
    if (kv.first == key) {
      b->seg = kv.second[0]; b->depth = kv.second[1]; b->ty = kv.second[2];
      b->sched = kv.second[3];
      b->tuned = true;
      return batch_tables(b);
    }
  hipEvent_t tb[2], tf[2];
  for (int q = 0; q < 2; q++) {
    (void)hipEventCreate(&tb[q]);
    (void)hipEventCreate(&tf[q]);
  }
  double best_b = 1e30, best_f = 1e30;
  int bseg = b->seg, bdep = b->depth, bty = b->ty;
  const int nseg = sizeof(kSegCand) / sizeof(int), nty = sizeof(kTyCand) / sizeof(int);
  const int ncand = std::max(nseg, nty);
  int rc = DMR_OK;
  b->sched = kSchedSeparate;
  for (int c = 0; c < ncand && !rc; c++) {
    b->seg = kSegCand[c % nseg];
    b->depth = stream_depth(b->seg);
    b->ty = kTyCand[c % nty];
    rc = batch_tables(b);
    float tbase = 0.f, tfine = 0.f;
    for (int rep = 0; rep < 2 && !rc; rep++) {  // two timed steps per candidate
      if (b->sims[0]->step - b->src_base >= kSrcSteps) rc = batch_sources(b, b->sims[0]->step);
      if (!rc) rc = batch_launch_step(b, tb, tf);
      if (!rc) (*used)++;
      if (!rc && hipStreamSynchronize(b->st) != hipSuccess) rc = DMR_EHIP;
      float x = 0.f, y = 0.f;
      (void)hipEventElapsedTime(&x, tb[0], tb[1]);
      (void)hipEventElapsedTime(&y, tf[0], tf[1]);
      tbase += x;
      tfine += y;
    }
    if (c < nseg && tbase < best_b) { best_b = tbase; bseg = b->seg; bdep = b->depth; }
    if (c < nty && tfine < best_f) { best_f = tfine; bty = b->ty; }
  }
  // the subcycle schedule: with the chosen streaming shape, time whole steps
  // of each schedule the instances allow (the patch tile height per
  // schedule) and keep the fastest
  int bsched = kSchedSeparate;
  b->seg = bseg; b->depth = bdep;
  auto step_ms = [&](int sched, int ty, float* ms) {
    b->sched = sched;
    b->ty = ty;
    int r = batch_tables(b);
    *ms = 0.f;
    for (int rep = 0; rep < 2 && !r; rep++) {
      if (b->sims[0]->step - b->src_base >= kSrcSteps) r = batch_sources(b, b->sims[0]->step);
      if (!r) r = batch_launch_step(b, tb, tf);
      if (!r) (*used)++;
      if (!r && hipStreamSynchronize(b->st) != hipSuccess) r = DMR_EHIP;
      float x = 0.f;
      (void)hipEventElapsedTime(&x, tb[0], tf[1]);
      *ms += x;
    }
    return r;
  };
  float best = 1e30f;
  if (!rc && (b->can_fuse || b->can_combine)) {
    float t = 0.f;
    rc = step_ms(kSchedSeparate, bty, &t);
    best = t;
    for (int sched = kSchedFused; sched <= kSchedCombined && !rc; sched++) {
      if ((sched == kSchedFused && !b->can_fuse) || (sched == kSchedCombined && !b->can_combine))
        continue;
      for (int c = 0; c < nty && !rc; c++) {
        rc = step_ms(sched, kTyCand[c], &t);
        if (!rc && t < best) { best = t; bsched = sched; bty = kTyCand[c]; }
      }
    }
  }
  for (int q = 0; q < 2; q++) {
    (void)hipEventDestroy(tb[q]);
    (void)hipEventDestroy(tf[q]);
  }
  if (rc) return rc;
  b->seg = bseg; b->depth = bdep; b->ty = bty; b->sched = bsched;
  b->tuned = true;
  tune_cache().push_back({key, {bseg, bdep, bty, bsched}});
  return batch_tables(b);
}

int batch_step(dmr_batch* b, int64_t n) {
  dmr_sim* s0 = b->sims[0];
  const dmr_params& p = s0->p;
  const bool dyn = p.mode == DMR_DYNAMIC;
  while (n > 0) {
    const int64_t step = s0->step;
    const int64_t base = step - step % kSrcSteps;
    int rc = DMR_OK;
    if (b->src_base != base) rc = batch_sources(b, base);
    if (rc) return rc;
    if (!b->tuned && !b->forced && step % kSrcSteps == 0 && n >= kSrcSteps &&
        (!dyn || p.regrid_every >= kSrcSteps)) {
      int64_t used = 0;
      rc = batch_tune(b, &used);  // times real steps of the run
      if (rc) return rc;
      n -= used;
      continue;
    }
    int64_t chunk = std::min<int64_t>(n, base + kSrcSteps - step);
    if (dyn) chunk = std::min<int64_t>(chunk, p.regrid_every - step % p.regrid_every);
    const bool steady = s0->blocks >= kRing || !p.continuity_on;
    const bool whole = step % kSrcSteps == 0 && chunk == kSrcSteps &&
                       (!dyn || p.regrid_every % kSrcSteps == 0);
    if (b->use_graph && whole && steady) {
      if (!b->graph_ok) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
          return bfail(b, DMR_EHIP, "graph capture begin");
        for (int q = 0; q < kSrcSteps && !rc; q++) rc = batch_launch_step(b, nullptr, nullptr);
        hipError_t e = hipStreamEndCapture(b->st, &g);
        if (rc) return rc;
        if (e != hipSuccess || hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess)
          return bfail(b, DMR_EHIP, "graph capture");
        (void)hipGraphDestroy(g);
        b->graph_ok = true;
        if (hipGraphLaunch(b->gexec, b->st) != hipSuccess) return bfail(b, DMR_EHIP, "graph launch");
      } else {
        if (hipGraphLaunch(b->gexec, b->st) != hipSuccess) return bfail(b, DMR_EHIP, "graph launch");
        int slot, update;
        for (int q = 0; q < kSrcSteps; q++) batch_advance(b, &slot, &update);
      }
    } else {
      for (int64_t q = 0; q < chunk && !rc; q++) rc = batch_launch_step(b, nullptr, nullptr);
      if (rc) return rc;
    }
    n -= chunk;
    if (dyn && s0->step % p.regrid_every == 0) {
      rc = batch_regrid(b);
      if (rc) return rc;
    }
  }
  return hipGetLastError() == hipSuccess ? DMR_OK : bfail(b, DMR_EHIP, "batch step");
}

}  // namespace

extern "C" {

int dmr_batch_workspace_bytes(const dmr_params* p, int count, size_t* bytes) {
  BatchLayout L;
  std::string why;
  const int rc = batch_layout(p, count, &L, &why);
  if (rc) return rc;
  if (!bytes) return DMR_EINVAL;
  *bytes = L.total;
  return DMR_OK;
}

int dmr_batch_create(const dmr_params* p, int count, const double* const* seed_base,
                     const double* const* seed_fine, void* d_workspace, size_t bytes,
                     void* stream, dmr_batch** out) {
  if (!out) return DMR_EINVAL;
  *out = nullptr;
  BatchLayout L;
  std::string why;
  int rc = batch_layout(p, count, &L, &why);
  if (rc) {
    fprintf(stderr, "dmr_batch_create: %s\n", why.c_str());
    return rc;
  }
  if (!d_workspace || bytes < L.total) return DMR_ENOMEM;
  dmr_batch* b = new (std::nothrow) dmr_batch();
  if (!b) return DMR_ENOMEM;
  b->count = count;
  b->user = (hipStream_t)stream;
  b->ws = (char*)d_workspace;
  if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&b->h_src, sizeof(float2) * kSrcSteps * count) != hipSuccess) {
    dmr_batch_destroy(b);
    return DMR_EHIP;
  }
  // the caller's earlier work (e.g. the workspace allocation) comes first
  (void)hipEventRecord(b->ev_in, b->user);
  (void)hipStreamWaitEvent(b->st, b->ev_in, 0);
  for (int k = 0; k < count; k++) {
    dmr_sim* s = nullptr;
    rc = dmr_create(&p[k], seed_base ? seed_base[k] : nullptr,
                    seed_fine ? seed_fine[k] : nullptr, b->ws + L.off[k], L.size[k], b->st, &s);
    if (rc) {
      dmr_batch_destroy(b);
      return rc;
    }
    s->fuse_fine = false;  // the batch's tables name fixed patch buffers
    s->combine = false;
    b->sims.push_back(s);
  }
  b->d_em = (EMArgs*)(b->ws + L.off_em);
  b->d_fem = (EMArgs*)(b->ws + L.off_fem);
  b->rf = L.rf;
  b->d_cont = (ContArgs*)(b->ws + L.off_cont);
  b->d_fcont = (ContArgs*)(b->ws + L.off_fcont);
  b->d_blk_base = (int2*)(b->ws + L.off_blk_base);
  b->d_blk_fine = (int2*)(b->ws + L.off_blk_fine);
  b->d_blk_cont = (int2*)(b->ws + L.off_blk_cont);
  b->d_blk_fcont = (int2*)(b->ws + L.off_blk_fcont);
  b->cap_base = std::max<size_t>(L.cap_base, 1); b->cap_fine = std::max<size_t>(L.cap_fine, 1);
  b->cap_cont = std::max<size_t>(L.cap_cont, 1); b->cap_fcont = std::max<size_t>(L.cap_fcont, 1);
  b->d_src = (float2*)(b->ws + L.off_src);
  b->d_fem2 = (EMArgs*)(b->ws + L.off_fem2);
  b->d_cem = (EMArgs*)(b->ws + L.off_cem);
  b->d_floc = (EMArgs*)(b->ws + L.off_floc);
  b->d_blk_comb = (int2*)(b->ws + L.off_blk_comb);
  b->cap_comb = std::max<size_t>(L.cap_comb, 1);
  rc = batch_tables(b);
  if (rc) {
    fprintf(stderr, "dmr_batch_create: %s\n", b->err.c_str());
    dmr_batch_destroy(b);
    return rc;
  }
  *out = b;
  return DMR_OK;
}

void dmr_batch_destroy(dmr_batch* b) {
  if (!b) return;
  if (b->st) (void)hipStreamSynchronize(b->st);
  for (dmr_sim* s : b->sims) dmr_destroy(s);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->h_src) (void)hipHostFree(b->h_src);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
}

int dmr_batch_step(dmr_batch* b, int64_t n) {
  if (!b || n < 0) return DMR_EINVAL;
  (void)hipEventRecord(b->ev_in, b->user);
  (void)hipStreamWaitEvent(b->st, b->ev_in, 0);
  const int rc = batch_step(b, n);
  (void)hipEventRecord(b->ev_out, b->st);
  (void)hipStreamWaitEvent(b->user, b->ev_out, 0);
  return rc;
}

int dmr_batch_instance(dmr_batch* b, int k, dmr_sim** out) {
  if (!b || !out || k < 0 || k >= b->count) return DMR_EINVAL;
  *out = b->sims[k];
  return DMR_OK;
}

int dmr_batch_sync(dmr_batch* b) {
  if (!b) return DMR_EINVAL;
  if (hipStreamSynchronize(b->st) != hipSuccess) return bfail(b, DMR_EHIP, "sync");
  for (dmr_sim* s : b->sims) {
    const int rc = dmr_sync(s);
    if (rc) return bfail(b, rc, s->err.c_str());
  }
  return DMR_OK;
}

int dmr_batch_config(dmr_batch* b, int32_t cfg[5]) {
  if (!b || !cfg) return DMR_EINVAL;
  cfg[0] = b->seg; cfg[1] = b->depth; cfg[2] = b->ty; cfg[3] = b->use_graph;
  cfg[4] = b->sched;
  return DMR_OK;
}

int dmr_batch_set_config(dmr_batch* b, const int32_t cfg[5]) {
  if (!b || !cfg || cfg[0] < 2 || (cfg[1] != 2 && cfg[1] != 4) ||
      (cfg[2] != 4 && cfg[2] != 8 && cfg[2] != 16) || cfg[4] < kSchedSeparate ||
      cfg[4] > kSchedCombined)
    return DMR_EINVAL;
  b->seg = cfg[0]; b->depth = cfg[1]; b->ty = cfg[2]; b->use_graph = cfg[3] != 0;
  b->sched = cfg[4];
  b->forced = true;
  int rc = batch_tables(b);
  if (!rc && b->sched != cfg[4])
    return bfail(b, DMR_EINVAL, "schedule not available for these instances (union levels: "
                                "separate only; combined: r = 2)");
  return rc;
}

const char* dmr_batch_last_error(const dmr_batch* b) {
  return b ? b->err.c_str() : "no handle";
}

}  // extern "C"
