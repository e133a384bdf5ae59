// dmr_api.hip -- host side of the C ABI in include/dmr.h: parameter checks,
// derived coefficients, workspace carving, the subcycling schedule of
// Sec. III.C and the regrid cadence of Sec. III.D.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dmr.h"
#include "dmr_kernels.h"

using namespace dmr;

namespace {

// CODATA 2018
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kPlanes = 21;  // Hz,Ex,Ey,Jx,Jy x2, n x2, acc, 8 window slots

struct Level {
  int NX = 0, NY = 0, pitch = 0;
  size_t plane = 0;
  float *hz[2] = {}, *ex[2] = {}, *ey[2] = {}, *jx[2] = {}, *jy[2] = {};
  float *n[2] = {}, *acc = nullptr, *ring = nullptr;
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
    off += align256(L.plane1 * kPlanes * sizeof(float));
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
  L.total = off;
  return L;
}

int check_params(const dmr_params* p, std::string* why) {
  auto bad = [&](const char* m) { *why = m; return DMR_EINVAL; };
  if (!p) return bad("params is NULL");
  if (p->struct_size != sizeof(dmr_params)) return bad("struct_size mismatch");
  if (p->nx < 4 || p->ny < 4) return bad("nx, ny must be >= 4");
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
  if (refined(p)) {
    if (p->r != 2) return bad("only r = 2 is supported");
    if (p->block < 2 || p->nx % p->block || p->ny % p->block)
      return bad("block must divide nx and ny");
    if (p->nx / p->block < 3 || p->ny / p->block < 3)
      return bad("need at least 3x3 blocks");
    if (p->mode == DMR_DYNAMIC &&
        (p->regrid_every <= 0 || p->regrid_every % (spp / kRing)))
      return bad("regrid_every must be a positive multiple of steps per window block");
    if (p->mode == DMR_STATIC) {
      const int* e = p->static_ext;
      if (e[0] < 1 || e[1] < 1 || e[2] > p->nx - 1 || e[3] > p->ny - 1 ||
          e[0] >= e[2] || e[1] >= e[3] || (p->tfsf_i > 0 && e[0] <= p->tfsf_i))
        return bad("static_ext outside the allowed region");
    }
  }
  return DMR_OK;
}

}  // namespace

struct dmr_sim {
  dmr_params p{};
  hipStream_t st = nullptr;
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
  uint8_t* d_flag = nullptr;
  int32_t *d_scan = nullptr, *d_list = nullptr;
  int* d_desc = nullptr;
  int* d_err = nullptr;
  float* stage = nullptr;
  int h_desc[16] = {};
  // timing
  bool timing = false;
  struct Ev { int cls; hipEvent_t a, b; };
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

void ev_begin(dmr_sim* s, int cls) {
  if (!s->timing) return;
  if (s->ev_used == s->evs.size()) {
    dmr_sim::Ev e{cls, nullptr, nullptr};
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
    s->evs.push_back(e);
  }
  s->evs[s->ev_used].cls = cls;
  (void)hipEventRecord(s->evs[s->ev_used].a, s->st);
}

void harvest(dmr_sim* s) {
  if (!s->ev_used) return;
  (void)hipStreamSynchronize(s->st);
  for (size_t k = 0; k < s->ev_used; k++) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->evs[k].a, s->evs[k].b) == hipSuccess) {
      s->t_ms[s->evs[k].cls] += ms;
      s->t_n[s->evs[k].cls] += 1;
    }
  }
  s->ev_used = 0;
}

void ev_end(dmr_sim* s) {
  if (!s->timing) return;
  (void)hipEventRecord(s->evs[s->ev_used].b, s->st);
  s->ev_used++;
  if (s->ev_used >= 4096) harvest(s);
}

// rows per segment of the streaming base kernel: long segments for
// bandwidth, short ones when the grid is too small to fill the chip
int stream_rows(int NX, int NY) {
  if (const char* e = getenv("DMR_SEG")) {
    const int v = atoi(e);
    if (v >= 2) return v;
  }
  const long waves_x = (NX + 1 + 61) / 62;
  int seg = 64;
  while (seg > 4 && waves_x * ((NY + seg) / seg) < 4096) seg >>= 1;
  return seg;
}

// rows in flight per wave: deep for short (latency-bound) segments
int stream_depth(int seg) {
  if (const char* e = getenv("DMR_DEPTH")) return atoi(e) >= 4 ? 4 : 2;
  return seg <= 8 ? 4 : 2;
}

int tile_rows(int NX, int NY) {
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

int regrid(dmr_sim* s, bool keep_n) {
  const dmr_params& p = s->p;
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

int base_step(dmr_sim* s) {
  Level &C = s->L0, &F = s->L1;
  const dmr_params& p = s->p;
  const int c = s->ccur;
  // coarse (or uniform) EM step n -> n+1
  EMArgs A{};
  em_args_level(&A, C, c, 1 - c, C.n[s->ncur], C.acc);
  A.L = 0; A.B = 0; A.R = p.nx; A.T = p.ny;
  A.bc_x = p.bc_x; A.bc_y = p.bc_y;
  A.is = p.tfsf_i;
  if (p.tfsf_i > 0) {
    const double t = (double)s->step * C.dt, xs = p.tfsf_i * C.dx;
    A.ey_src = (float)ey_inc(s, xs, t);
    A.hz_src = (float)ey_inc(s, xs - 0.5 * C.dx, t + 0.5 * C.dt);
  }
  ev_begin(s, 0);
  hipError_t e = launch_em_stream(A, s->seg0, s->depth0, s->st);
  ev_end(s);
  if (e != hipSuccess) return hipfail(s, e, "base EM launch");
  if (s->has_patch) {  // two fine substeps (Sec. III.C)
    const int r = p.r;
    for (int m = 1; m <= r; m++) {
      EMArgs G{};
      const int src = (m - 1) & 1, dst = m & 1;
      em_args_level(&G, F, src, dst, F.n[s->ncur], F.acc);
      G.L = r * s->ext[0]; G.B = r * s->ext[1];
      G.R = r * s->ext[2]; G.T = r * s->ext[3];
      G.cex0 = C.ex[c]; G.cey0 = C.ey[c];
      G.cex1 = C.ex[1 - c]; G.cey1 = C.ey[1 - c];
      G.cpitch = C.pitch;
      G.frac = (float)m / (float)r;
      G.gamma = (float)p.fine_filter;
      if (m == r) {
        G.restrict_on = 1;
        G.chz = C.hz[1 - c]; G.cex = C.ex[1 - c]; G.cey = C.ey[1 - c];
        G.cjx = C.jx[1 - c]; G.cjy = C.jy[1 - c];
      }
      ev_begin(s, 1);
      e = launch_em(G, true, s->ty1, s->st);
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "fine EM launch");
    }
  }
  s->ccur = 1 - c;
  s->step++;
  if (p.continuity_on && s->step % C.spb == 0) {
    const int slot = (int)(s->blocks % kRing);
    s->blocks++;
    const int update = s->blocks >= kRing;
    ContArgs K{};
    K.n0 = C.n[s->ncur]; K.n1 = C.n[1 - s->ncur];
    K.acc = C.acc; K.ring = C.ring; K.plane = C.plane; K.pitch = C.pitch;
    K.L = 0; K.B = 0; K.R = p.nx; K.T = p.ny;
    K.slot = slot; K.update = update;
    K.inv_spp = (float)(1.0 / C.spp);
    K.dtn = (float)(C.spb * C.dt);
    K.inv_dx2 = (float)(1.0 / (C.dx * C.dx));
    K.eeff_p2 = (float)(s->eeff / (1.0e4 * p.p_torr * p.p_torr));
    K.half_beta = (float)(0.5 * p.beta_ion);
    K.att = (float)std::pow(p.ecr_over_p, p.beta_ion);
    K.nuA = (float)(s->nu_m * p.A_ion);
    K.inv_namb = (float)(1.0 / s->n_amb);
    K.De = (float)s->De; K.Da = (float)s->Da;
    K.d_const_mode = p.d_mode == DMR_D_CONST;
    K.d_const = (float)p.d_const;
    K.err = s->d_err;
    ev_begin(s, 2);
    e = launch_cont(K, false, s->st);
    ev_end(s);
    if (e != hipSuccess) return hipfail(s, e, "continuity launch");
    if (s->has_patch) {
      ContArgs G = K;
      G.n0 = F.n[s->ncur]; G.n1 = F.n[1 - s->ncur];
      G.acc = F.acc; G.ring = F.ring; G.plane = F.plane; G.pitch = F.pitch;
      G.L = p.r * s->ext[0]; G.B = p.r * s->ext[1];
      G.R = p.r * s->ext[2]; G.T = p.r * s->ext[3];
      G.inv_spp = (float)(1.0 / F.spp);
      G.dtn = (float)(F.spb * F.dt);
      G.inv_dx2 = (float)(1.0 / (F.dx * F.dx));
      G.cn1 = C.n[1 - s->ncur]; G.cpitch = C.pitch;
      ev_begin(s, 2);
      e = launch_cont(G, true, s->st);
      ev_end(s);
      if (e != hipSuccess) return hipfail(s, e, "fine continuity launch");
    }
    if (update) s->ncur = 1 - s->ncur;
  }
  if (p.mode == DMR_DYNAMIC && s->step % p.regrid_every == 0)
    return regrid(s, false);
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
  derive(s);
  const double dx0 = s->lambda / p->cells_per_lambda;
  const double dt0 = p->courant * dx0 / kC0;
  const int spp0 = (int)std::lround(p->cells_per_lambda / p->courant);
  // numerical wavenumber of the 1-D Yee wave
  s->ktil = 2.0 / dx0 * std::asin(std::sin(0.5 * s->omega * dt0) / p->courant);
  carve(s, &s->L0, 0, lay.plane0, lay.pitch0, p->nx, p->ny);
  level_coeffs(s, &s->L0, dx0, dt0, spp0);
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
  s->seg0 = stream_rows(p->nx, p->ny);
  s->depth0 = stream_depth(s->seg0);
  hipError_t e = hipMemsetAsync(s->ws, 0, lay.total, s->st);
  if (e != hipSuccess) { rc = hipfail(s, e, "workspace clear"); delete s; return rc; }
  // seeds: float32 on the pitched node grid
  std::vector<float> h;
  auto upload = [&](const double* src, const Level& L) -> hipError_t {
    h.assign(L.plane, 0.f);
    for (int j = 0; j <= L.NY; j++)
      for (int i = 0; i <= L.NX; i++)
        h[(size_t)j * L.pitch + i] = (float)src[(size_t)j * (L.NX + 1) + i];
    hipError_t r1 = hipMemcpyAsync(L.n[0], h.data(), L.plane * sizeof(float),
                                   hipMemcpyHostToDevice, s->st);
    if (r1 != hipSuccess) return r1;
    return hipStreamSynchronize(s->st);
  };
  if (seed_base && (e = upload(seed_base, s->L0)) != hipSuccess) {
    rc = hipfail(s, e, "seed upload");
    delete s;
    return rc;
  }
  const bool keep_n = refined(p) && seed_fine;
  if (keep_n && (e = upload(seed_fine, s->L1)) != hipSuccess) {
    rc = hipfail(s, e, "fine seed upload");
    delete s;
    return rc;
  }
  if (p->mode == DMR_STATIC) rc = prolong(s, p->static_ext, keep_n);
  else if (p->mode == DMR_DYNAMIC) rc = regrid(s, keep_n);
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
    if (rc) return rc;
  }
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
