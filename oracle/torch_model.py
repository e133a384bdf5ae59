"""FP64 PyTorch-CPU model of the refined update, for the reference adjoint.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).  A second plain
implementation of the same discrete update as dmr_oracle.c (Eqs. (1)-(5),
Sec. II-III), written with whole-array torch operations in float64 so that
torch.autograd yields the exact discrete adjoint of the objective
F = dx_c^2 * sum_w w * n_c(t_final) with respect to the incident amplitude
E0, the ionisation coefficients A and beta and the coarse seed density
(power-law source; with the Townsend source of Eq. (4) A and beta do not
enter and their gradients are zero; recombination is included in both).
The forward is checked against the C oracle (test_oracle_adjoint.py); the
gradients against central finite differences of the C oracle.

Scope: uniform runs and refined runs.  The patch extents over time are
given (the regrid decisions are integer and have no derivative): the patch
present at t = 0 and a schedule of growths, each applied after the base step
that ends on a regrid point, as the forward run decided them.  The fine seed
and every newly covered fine entity are the Eq. (5a) prolongation of the
coarse data (Sec. III.D).
"""
from __future__ import annotations

import math

import torch
from torch.utils.checkpoint import checkpoint

QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
C0 = 299792458.0
MU0 = 1.0 / (EPS0 * C0 * C0)
KB = 1.380649e-23


def derived(cfg):
    w = 2 * math.pi * cfg["freq_hz"]
    lam = C0 / cfg["freq_hz"]
    num = 5.3e9 * cfg["p_torr"]
    eeff = 1.0 / (1.0 + (w / num) ** 2)
    ecr = cfg["ecr_over_p"] * 100.0 * cfg["p_torr"]
    e0 = math.sqrt(2.0) * cfg["erms_over_ebd"] * ecr / math.sqrt(eeff)
    dx = lam / cfg["cells_per_lambda"]
    dt = cfg["courant"] * dx / C0
    ktil = 2.0 / dx * math.asin(math.sin(0.5 * w * dt) / cfg["courant"])
    d = dict(omega=w, lam=lam, nu_m=num, eeff=eeff, E0=e0, dx=dx, dt=dt, ktil=ktil,
             n_c=ME * EPS0 * w * w / QE ** 2,
             De=QE * cfg["te_ev"] / (ME * num),
             Da=cfg["mu_i_760"] * (760.0 / cfg["p_torr"]) * (cfg["te_ev"] + cfg["ti_ev"]),
             n_amb=EPS0 * cfg["te_ev"] / (QE * cfg["L_amb"] ** 2),
             spp=int(round(cfg["cells_per_lambda"] / cfg["courant"])))
    # recombination coefficient of Eq. (4), m^3/s, with T_e in kelvin
    brec = cfg.get("beta_rec", 0.0)
    d["r_ei"] = brec * 1e-13 * math.sqrt(300.0 / (cfg["te_ev"] * QE / KB)) if brec > 0 else 0.0
    return d


def unit_incident(cfg, d, steps, dx, dt):
    """Incident Ey at the source line (t^n) and at x_s - dx/2 (t^{n+1/2}),
    for unit amplitude: g(t - x/c) sin(w t - k~ x)."""
    tr = cfg["ramp_periods"] / cfg["freq_hz"]
    xs = cfg["tfsf_i"] * dx

    def f(x, t):
        tau = t - x / C0
        g = 0.0 if tau <= 0 else (1.0 if tau >= tr else math.sin(0.5 * math.pi * tau / tr) ** 2)
        return g * math.sin(d["omega"] * t - d["ktil"] * x)

    ey = torch.tensor([f(xs, n * dt) for n in range(steps)], dtype=torch.float64)
    hz = torch.tensor([f(xs - 0.5 * dx, (n + 0.5) * dt) / (MU0 * C0) for n in range(steps)],
                      dtype=torch.float64)
    return ey, hz


class Level:
    """Coefficients of one level."""

    def __init__(self, d, dx, dt, spp):
        self.dx, self.dt, self.spp, self.spb = dx, dt, spp, spp // 8
        self.ch = dt / (MU0 * dx)
        self.ce = dt / EPS0
        self.a = math.exp(-d["nu_m"] * dt)
        self.b = QE * QE * (1.0 - self.a) / (ME * d["nu_m"])
        self.kn = dt * self.b / (4.0 * EPS0)
        S = C0 * dt / dx
        self.cmur = (S - 1.0) / (S + 1.0)


def _ej(L, e, j, curl, ne):
    kap = L.kn * ne
    en = ((1.0 - kap) * e + L.ce * (curl - 0.5 * (1.0 + L.a) * j)) / (1.0 + kap)
    jn = L.a * j + 0.5 * L.b * ne * (e + en)
    return en, jn


def _node_e2(ex, ey):
    """Mean of the squares of the existing edges per axis, at the nodes of a
    rectangle (Ex [ny+1][nx], Ey [ny][nx+1])."""
    ex2, ey2 = ex * ex, ey * ey
    sx = torch.zeros(ex.shape[0], ex.shape[1] + 1, dtype=ex.dtype)
    sx = sx + torch.nn.functional.pad(ex2, (1, 0)) + torch.nn.functional.pad(ex2, (0, 1))
    cx = torch.full((ex.shape[1] + 1,), 2.0, dtype=ex.dtype)
    cx[0] = cx[-1] = 1.0
    sy = torch.nn.functional.pad(ey2, (0, 0, 1, 0)) + torch.nn.functional.pad(ey2, (0, 0, 0, 1))
    cy = torch.full((ey.shape[0] + 1, 1), 2.0, dtype=ey.dtype)
    cy[0] = cy[-1] = 1.0
    return sx / cx + sy / cy


def _lap_rep(a):
    """5-point Laplacian with each outside neighbour replaced by the entry."""
    p = torch.nn.functional.pad(a[None, None], (1, 1, 1, 1), mode="replicate")[0, 0]
    return p[1:-1, :-2] + p[1:-1, 2:] + p[:-2, 1:-1] + p[2:, 1:-1] - 4.0 * a


def _bilin(arr, U4, V4):
    """Bilinear sample of a [rows][cols] array at quarter-unit positions."""
    i = U4 // 4
    j = V4 // 4
    fu = (U4 % 4).to(torch.float64) / 4.0
    fv = (V4 % 4).to(torch.float64) / 4.0
    i1 = torch.clamp(i + 1, max=arr.shape[1] - 1)
    j1 = torch.clamp(j + 1, max=arr.shape[0] - 1)
    return ((1 - fu) * (1 - fv) * arr[j, i] + fu * (1 - fv) * arr[j, i1] +
            (1 - fu) * fv * arr[j1, i] + fu * fv * arr[j1, i1])


class Model:
    """One run with parameters (scale of E0, A, beta) and a coarse seed."""

    def __init__(self, cfg, ext=None, growth=None):
        """ext: patch at t = 0 (coarse cells I0, J0, I1, J1) or None;
        growth: {base steps completed: new ext} for the growths of the run."""
        assert cfg["mode"] in ("uniform", "static", "dynamic")
        assert cfg["bc_x"] == "mur" and cfg["bc_y"] == "mur"
        self.cfg = cfg
        self.d = derived(cfg)
        d = self.d
        self.L0 = Level(d, d["dx"], d["dt"], d["spp"])
        self.refined = cfg["mode"] != "uniform"
        self.ext = tuple(ext) if (self.refined and ext is not None) else None
        if self.ext is not None and self.ext[2] <= self.ext[0]:
            self.ext = None
        self.growth = {int(k): tuple(v) for k, v in (growth or {}).items()} if self.refined else {}
        self.L1 = Level(d, d["dx"] / 2, d["dt"] / 2, 2 * d["spp"])

    def ext_at(self, k):
        """Patch extents during base step k (after the growths of steps <= k)."""
        e = self.ext
        for q in sorted(self.growth):
            if q <= k:
                e = self.growth[q]
        return e

    # ---- ionisation and diffusion (Eq. (4), Sec. II.A) ------------------
    def nu(self, e2, A, beta):
        """Net ionisation rate of Eq. (4) at E_rms^2 = e2: the power law in
        E_eff/p (coefficients A, beta), or Townsend's gamma v_d minus a
        constant attachment rate (then A and beta do not enter)."""
        c = self.cfg
        if c.get("source_model", "power") == "townsend":
            eeff = torch.sqrt(torch.clamp(e2 * self.d["eeff"], min=1e-300))   # V/m
            pos = e2 > 0
            e_cm = eeff / 100.0
            gamma_cm = c["A_town"] * c["p_torr"] * torch.exp(-c["B_town"] * c["p_torr"] / e_cm)
            v_d = QE / (ME * self.d["nu_m"]) * eeff
            return torch.where(pos, 100.0 * gamma_cm * v_d, torch.zeros_like(e2)) - c["nu_att"]
        x = e2 * self.d["eeff"] / (1e4 * c["p_torr"] ** 2)
        xb = torch.where(x > 0, torch.pow(torch.clamp(x, min=1e-300), 0.5 * beta),
                         torch.zeros_like(x))
        cb = torch.pow(torch.tensor(c["ecr_over_p"], dtype=torch.float64), beta)
        return self.d["nu_m"] * A * (xb - cb)

    def deff(self, n):
        al = n / self.d["n_amb"]
        return (al * self.d["Da"] + self.d["De"]) / (1.0 + al)

    def continuity(self, L, n, e2, A, beta, interior):
        """Forward Euler flux form; zero-flux outer faces or (interior) the
        boundary ring left unchanged."""
        dtn = L.spb * L.dt
        D = self.deff(n)
        fx = 0.5 * (D[:, 1:] + D[:, :-1]) * (n[:, 1:] - n[:, :-1])   # face i+1/2
        fy = 0.5 * (D[1:, :] + D[:-1, :]) * (n[1:, :] - n[:-1, :])
        flux = torch.zeros_like(n)
        flux = flux + torch.nn.functional.pad(fx, (0, 1)) - torch.nn.functional.pad(fx, (1, 0))
        flux = flux + torch.nn.functional.pad(fy, (0, 0, 0, 1)) - torch.nn.functional.pad(fy, (0, 0, 1, 0))
        nn = n + dtn * (flux / (L.dx * L.dx) + self.nu(e2, A, beta) * n - self.d["r_ei"] * n * n)
        nn = torch.clamp(nn, min=0.0)
        if interior:
            out = n.clone()
            out[1:-1, 1:-1] = nn[1:-1, 1:-1]
            return out
        return nn

    # ---- EM steps ---------------------------------------------------------
    def em_base(self, st, ey_s, hz_s):
        L = self.L0
        hz, ex, ey, jx, jy, n = st["hz"], st["ex"], st["ey"], st["jx"], st["jy"], st["n"]
        i_s = self.cfg["tfsf_i"]
        hz = hz - L.ch * ((ey[:, 1:] - ey[:, :-1]) - (ex[1:, :] - ex[:-1, :]))
        hz = hz + L.ch * ey_s * torch.nn.functional.one_hot(
            torch.tensor(i_s - 1), hz.shape[1]).to(torch.float64)[None, :]
        # interior Ex (rows 1..ny-1), Ey (cols 1..nx-1)
        curlx = (hz[1:, :] - hz[:-1, :]) / L.dx
        nex = 0.5 * (n[1:-1, :-1] + n[1:-1, 1:])
        exi, jxi = _ej(L, ex[1:-1, :], jx[1:-1, :], curlx, nex)
        curly = -(hz[:, 1:] - hz[:, :-1]) / L.dx
        src = torch.zeros(hz.shape[1] - 1, dtype=torch.float64)
        src[i_s - 1] = 1.0
        curly = curly + (hz_s / L.dx) * src[None, :]
        ney = 0.5 * (n[:-1, 1:-1] + n[1:, 1:-1])
        eyi, jyi = _ej(L, ey[:, 1:-1], jy[:, 1:-1], curly, ney)
        # Mur on tangential edges (old values from the step input)
        cm = L.cmur
        ey_l = ey[:, 1] + cm * (eyi[:, 0] - ey[:, 0])
        ey_r = ey[:, -2] + cm * (eyi[:, -1] - ey[:, -1])
        ex_b = ex[1, :] + cm * (exi[0, :] - ex[0, :])
        ex_t = ex[-2, :] + cm * (exi[-1, :] - ex[-1, :])
        ne_l = 0.5 * (n[:-1, 0] + n[1:, 0])
        ne_r = 0.5 * (n[:-1, -1] + n[1:, -1])
        ne_b = 0.5 * (n[0, :-1] + n[0, 1:])
        ne_t = 0.5 * (n[-1, :-1] + n[-1, 1:])
        jy_l = L.a * jy[:, 0] + 0.5 * L.b * ne_l * (ey[:, 0] + ey_l)
        jy_r = L.a * jy[:, -1] + 0.5 * L.b * ne_r * (ey[:, -1] + ey_r)
        jx_b = L.a * jx[0, :] + 0.5 * L.b * ne_b * (ex[0, :] + ex_b)
        jx_t = L.a * jx[-1, :] + 0.5 * L.b * ne_t * (ex[-1, :] + ex_t)
        ey_n = torch.cat([ey_l[:, None], eyi, ey_r[:, None]], 1)
        jy_n = torch.cat([jy_l[:, None], jyi, jy_r[:, None]], 1)
        ex_n = torch.cat([ex_b[None, :], exi, ex_t[None, :]], 0)
        jx_n = torch.cat([jx_b[None, :], jxi, jx_t[None, :]], 0)
        out = dict(st)
        out.update(hz=hz, ex=ex_n, ey=ey_n, jx=jx_n, jy=jy_n, acc=st["acc"] + _node_e2(ex_n, ey_n))
        return out

    def em_fine(self, fs, ex_old, ey_old, ex_new, ey_new, m, gamma, ext):
        """One fine substep; coarse E before/after the coarse step for the
        boundary (Eq. (5b))."""
        L = self.L1
        I0, J0, I1, J1 = ext
        hz, ex, ey, jx, jy, n = fs["hz"], fs["ex"], fs["ey"], fs["jx"], fs["jy"], fs["n"]
        if gamma > 0:
            dx_ = gamma * _lap_rep(_lap_rep(ex))
            ex = torch.cat([ex[:1], ex[1:-1] - dx_[1:-1], ex[-1:]], 0)
            dy_ = gamma * _lap_rep(_lap_rep(ey))
            ey = torch.cat([ey[:, :1], ey[:, 1:-1] - dy_[:, 1:-1], ey[:, -1:]], 1)
        hz = hz - L.ch * ((ey[:, 1:] - ey[:, :-1]) - (ex[1:, :] - ex[:-1, :]))
        curlx = (hz[1:, :] - hz[:-1, :]) / L.dx
        exi, jxi = _ej(L, ex[1:-1, :], jx[1:-1, :], curlx, 0.5 * (n[1:-1, :-1] + n[1:-1, 1:]))
        curly = -(hz[:, 1:] - hz[:, :-1]) / L.dx
        eyi, jyi = _ej(L, ey[:, 1:-1], jy[:, 1:-1], curly, 0.5 * (n[:-1, 1:-1] + n[1:, 1:-1]))
        frac = m / 2.0
        fh, fw = hz.shape
        # fine y-edges on x = I0, I1: coarse Ey column, rows by quarter units
        Q = torch.arange(fh) + 2 * J0
        V4 = 2 * Q - 1

        def line_y(arr, I):
            j = V4 // 4
            f = (V4 % 4).to(torch.float64) / 4.0
            return (1 - f) * arr[j, I] + f * arr[j + 1, I]

        P = torch.arange(fw) + 2 * I0
        U4 = 2 * P - 1

        def line_x(arr, J):
            i = U4 // 4
            f = (U4 % 4).to(torch.float64) / 4.0
            return (1 - f) * arr[J, i] + f * arr[J, i + 1]

        eb = [(1 - frac) * line_y(ey_old, I) + frac * line_y(ey_new, I) for I in (I0, I1)]
        xb = [(1 - frac) * line_x(ex_old, J) + frac * line_x(ex_new, J) for J in (J0, J1)]
        ne_l = 0.5 * (n[:-1, 0] + n[1:, 0])
        ne_r = 0.5 * (n[:-1, -1] + n[1:, -1])
        ne_b = 0.5 * (n[0, :-1] + n[0, 1:])
        ne_t = 0.5 * (n[-1, :-1] + n[-1, 1:])
        jy_l = L.a * jy[:, 0] + 0.5 * L.b * ne_l * (ey[:, 0] + eb[0])
        jy_r = L.a * jy[:, -1] + 0.5 * L.b * ne_r * (ey[:, -1] + eb[1])
        jx_b = L.a * jx[0, :] + 0.5 * L.b * ne_b * (ex[0, :] + xb[0])
        jx_t = L.a * jx[-1, :] + 0.5 * L.b * ne_t * (ex[-1, :] + xb[1])
        ey_n = torch.cat([eb[0][:, None], eyi, eb[1][:, None]], 1)
        jy_n = torch.cat([jy_l[:, None], jyi, jy_r[:, None]], 1)
        ex_n = torch.cat([xb[0][None, :], exi, xb[1][None, :]], 0)
        jx_n = torch.cat([jx_b[None, :], jxi, jx_t[None, :]], 0)
        out = dict(fs)
        out.update(hz=hz, ex=ex_n, ey=ey_n, jx=jx_n, jy=jy_n, acc=fs["acc"] + _node_e2(ex_n, ey_n))
        return out

    def restrict(self, cs, hz1, fs, ext):
        I0, J0, I1, J1 = ext
        h = 0.5 * (hz1 + fs["hz"])
        hr = 0.25 * (h[0::2, 0::2] + h[0::2, 1::2] + h[1::2, 0::2] + h[1::2, 1::2])
        hz = cs["hz"].clone()
        hz[J0:J1, I0:I1] = hr
        ex, jx, ey, jy = cs["ex"].clone(), cs["jx"].clone(), cs["ey"].clone(), cs["jy"].clone()
        ex[J0 + 1:J1, I0:I1] = 0.5 * (fs["ex"][2:-1:2, 0::2] + fs["ex"][2:-1:2, 1::2])
        jx[J0 + 1:J1, I0:I1] = 0.5 * (fs["jx"][2:-1:2, 0::2] + fs["jx"][2:-1:2, 1::2])
        ey[J0:J1, I0 + 1:I1] = 0.5 * (fs["ey"][0::2, 2:-1:2] + fs["ey"][1::2, 2:-1:2])
        jy[J0:J1, I0 + 1:I1] = 0.5 * (fs["jy"][0::2, 2:-1:2] + fs["jy"][1::2, 2:-1:2])
        out = dict(cs)
        out.update(hz=hz, ex=ex, jx=jx, ey=ey, jy=jy)
        return out

    def sync(self, cs, fs, blocks, A, beta, ext):
        """Window block close, continuity on both levels, density transfers."""
        slot = blocks % 8

        def close(s, L):
            ring = s["ring"].clone()
            ring[slot] = s["acc"] / L.spp
            s = dict(s)
            s.update(ring=ring, acc=torch.zeros_like(s["acc"]))
            return s

        cs = close(cs, self.L0)
        if fs is not None:
            fs = close(fs, self.L1)
        blocks += 1
        if blocks < 8:
            return cs, fs, blocks
        cs = dict(cs)
        cs["n"] = self.continuity(self.L0, cs["n"], cs["ring"].sum(0), A, beta, False)
        if fs is not None:
            fs = dict(fs)
            nf = self.continuity(self.L1, fs["n"], fs["ring"].sum(0), A, beta, True)
            I0, J0, I1, J1 = ext
            nc = cs["n"]
            # boundary nodes from the new coarse density (copy / mean)
            edge = nc[J0:J1 + 1, I0:I1 + 1]
            up = torch.zeros(2 * (J1 - J0) + 1, 2 * (I1 - I0) + 1, dtype=torch.float64)
            up[0::2, 0::2] = edge
            up[0::2, 1::2] = 0.5 * (edge[:, :-1] + edge[:, 1:])
            up[1::2, 0::2] = 0.5 * (edge[:-1, :] + edge[1:, :])
            mask = torch.zeros_like(nf, dtype=torch.bool)
            mask[0, :] = mask[-1, :] = True
            mask[:, 0] = mask[:, -1] = True
            nf = torch.where(mask, up, nf)
            fs["n"] = nf
            nc = nc.clone()
            nc[J0 + 1:J1, I0 + 1:I1] = nf[2:-1:2, 2:-1:2]
            cs["n"] = nc
        return cs, fs, blocks

    # ---- initial state -----------------------------------------------------
    def initial(self, seed):
        c = self.cfg
        ny, nx = c["ny"], c["nx"]
        z = lambda r, q: torch.zeros(r, q, dtype=torch.float64)
        cs = dict(hz=z(ny, nx), ex=z(ny + 1, nx), ey=z(ny, nx + 1), jx=z(ny + 1, nx),
                  jy=z(ny, nx + 1), n=seed, acc=z(ny + 1, nx + 1),
                  ring=torch.zeros(8, ny + 1, nx + 1, dtype=torch.float64))
        fs = None
        if self.ext is not None:   # Eq. (5a): fine seed from the coarse seed
            fs = self.grow(cs, None, cs["hz"], None, self.ext)
        return cs, fs

    def grow(self, cs, fs, hz_prev, old, new):
        """New patch `new`: entities of the old patch keep their values, the
        others are the Eq. (5a) bilinear prolongation of the coarse data at
        the current coarse time; Hz at 5/4 of the way from the coarse
        Hz^{n-1/2} (hz_prev) to Hz^{n+1/2}, where fine Hz lives."""
        I0, J0, I1, J1 = new
        fw, fh = 2 * (I1 - I0), 2 * (J1 - J0)
        P = torch.arange(fw + 1) + 2 * I0
        Q = torch.arange(fh + 1) + 2 * J0

        def grid(rows, cols, du, dv):
            # quarter-unit positions: 2P (+du) across, 2Q (+dv) up
            U4 = (2 * P[:cols] + du)[None, :].expand(rows, -1)
            V4 = (2 * Q[:rows] + dv)[:, None].expand(-1, cols)
            return U4, V4

        def keep(rows, cols, hx, hy):
            m = torch.zeros(rows, cols, dtype=torch.bool)
            if fs is None:
                return m, None
            oI0, oJ0, oI1, oJ1 = old
            pp, qq = P[:cols], Q[:rows]
            inx = (pp >= 2 * oI0) & (pp <= 2 * oI1 - hx)
            iny = (qq >= 2 * oJ0) & (qq <= 2 * oJ1 - hy)
            m = iny[:, None] & inx[None, :]
            return m, (2 * (oI0 - I0), 2 * (oJ0 - J0))

        def place(new_val, key, hx, hy):
            rows, cols = new_val.shape[-2:]
            m, off = keep(rows, cols, hx, hy)
            if off is None:
                return new_val
            old_val = fs[key]
            pad = torch.zeros_like(new_val)
            r0, c0 = off[1], off[0]
            pad[..., r0:r0 + old_val.shape[-2], c0:c0 + old_val.shape[-1]] = old_val
            return torch.where(m, pad, new_val)

        out = {}
        U, V = grid(fh, fw, -1, -1)
        h = -0.25 * _bilin(hz_prev, U, V) + 1.25 * _bilin(cs["hz"], U, V)
        out["hz"] = place(h, "hz", 1, 1)
        U, V = grid(fh + 1, fw, -1, 0)
        out["ex"] = place(_bilin(cs["ex"], U, V), "ex", 1, 0)
        out["jx"] = place(_bilin(cs["jx"], U, V), "jx", 1, 0)
        U, V = grid(fh, fw + 1, 0, -1)
        out["ey"] = place(_bilin(cs["ey"], U, V), "ey", 0, 1)
        out["jy"] = place(_bilin(cs["jy"], U, V), "jy", 0, 1)
        U, V = grid(fh + 1, fw + 1, 0, 0)
        out["n"] = place(_bilin(cs["n"], U, V), "n", 0, 0)
        out["acc"] = place(_bilin(cs["acc"], U, V), "acc", 0, 0)
        out["ring"] = place(torch.stack([_bilin(cs["ring"][q], U, V) for q in range(8)]),
                            "ring", 0, 0)
        return out

    # ---- run ---------------------------------------------------------------
    def run(self, seed, e0_scale, A, beta, steps, seg=45, grad=True):
        """Advance `steps` base steps; returns the final coarse and fine
        states.  e0_scale multiplies the incident amplitude of cfg."""
        d = self.d
        f64 = lambda v: torch.as_tensor(v, dtype=torch.float64)
        seed, e0_scale, A, beta = f64(seed), f64(e0_scale), f64(A), f64(beta)
        ey_u, hz_u = unit_incident(self.cfg, d, steps, d["dx"], d["dt"])
        cs, fs = self.initial(seed)
        gamma = self.cfg["fine_filter"]
        E0 = e0_scale * d["E0"]
        keys = ["hz", "ex", "ey", "jx", "jy", "n", "acc", "ring"]

        def segment(k0, k1, blocks, *flat):
            c = dict(zip(keys, flat[:8]))
            f = dict(zip(keys, flat[8:])) if len(flat) > 8 else None
            ext = self.ext_at(k0)
            for k in range(k0, k1):
                ex_old, ey_old, hz_prev = c["ex"], c["ey"], c["hz"]
                c = self.em_base(c, E0 * ey_u[k], E0 * hz_u[k])
                if f is not None:
                    f1 = self.em_fine(f, ex_old, ey_old, c["ex"], c["ey"], 1, gamma, ext)
                    f = self.em_fine(f1, ex_old, ey_old, c["ex"], c["ey"], 2, gamma, ext)
                    c = self.restrict(c, f1["hz"], f, ext)
                if self.cfg["continuity_on"] and (k + 1) % self.L0.spb == 0:
                    c, f, blocks = self.sync(c, f, blocks, A, beta, ext)
                if (k + 1) in self.growth:
                    new = self.growth[k + 1]
                    f = self.grow(c, f, hz_prev, ext, new)
                    ext = new
            out = [c[k] for k in keys] + ([f[k] for k in keys] if f is not None else [])
            return tuple(out)

        blocks = 0
        flat = tuple([cs[k] for k in keys] + ([fs[k] for k in keys] if fs is not None else []))
        k = 0
        while k < steps:
            k1 = min(steps, k + seg)
            nblk = sum(1 for q in range(k, k1)
                       if self.cfg["continuity_on"] and (q + 1) % self.L0.spb == 0)
            b0 = blocks
            if grad:
                flat = checkpoint(lambda *x, k=k, k1=k1, b0=b0: segment(k, k1, b0, *x),
                                  *flat, use_reentrant=False)
            else:
                flat = segment(k, k1, b0, *flat)
            blocks += nblk
            k = k1
        cs = dict(zip(keys, flat[:8]))
        fs = dict(zip(keys, flat[8:])) if len(flat) > 8 else None
        return cs, fs
