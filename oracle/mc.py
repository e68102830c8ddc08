"""The Monte Carlo QED step, in float64, in particle-index order
(test infrastructure only).

The paper's event generator (text after Eq. 7; method II, the cumulative
probability 1 - exp(-P_cum) > r_3) is written as an optical depth: each particle
carries tau = -ln(r), tau is decremented by W dt, and an event fires when it is
exhausted.  The overshoot is carried: when tau <= W * rem inside a step, the
event happens after tau / W of the remaining time, a new tau is drawn, and the
rest of the step is spent with the (possibly changed) rate.  At most KMAX
events per particle and step; a particle that reaches the cap carries a
negative tau into the next step.  Method I (emit if W Dt > r_1, at most one
event per step) is kept as ``lepton_step_method1`` for the paper's time-step
study.

Per lepton (``lepton_step``):
  1. Boris push with E, B at x^n (charge q = -1 electron, +1 positron)
  2. x^{n+1} = x^n + p/gamma dt (periodic wrap if a box length is given)
  3. chi_e from Eq. (2) with the same E, B and p^{n+1/2}
  4. W = alpha E_S h(chi) / gamma (uncut rate)
  5. optical-depth loop; per event k: draw (u_xi, u_tau, u_row, u_ph) from the
     particle's stream; xi from the inverse CDF (Eq. 7); if xi gamma >= 2 (the
     infrared cutoff xi_min eps_e = 2 m_e c^2) a photon of energy xi gamma is
     emitted along p with tau_ph = -ln u_ph, and the lepton recoils to
     gamma' = max((1 - xi) gamma, 1) along the same direction (the energies the
     paper defines); otherwise nothing is emitted (thinning); tau = -ln u_tau.
  6. appended photons are ordered by (parent index, k); ids = next_id + rank.

Per photon (``photon_step``):
  optional ballistic move; chi_ph from Eq. (3); W_pair = alpha E_S h_pair / gamma_ph
  (0 below gamma_ph = 2); on an event xi = eps_e / eps_ph is drawn from the
  symmetric half-spectrum and exchanged with 1 - xi by one random bit; the
  electron gets xi gamma_ph and the positron the rest (text under Eq. 6), both
  along the photon direction; the photon is marked dead.  Pairs are appended
  in parent order; the electron and positron of one pair share the rank r and
  get ids next_id + 2r and next_id + 2r + 1.

``compact`` keeps the live particles in order (exclusive prefix sum of the
alive flags).

Pinned by tests/test_oracle_mc.py: Poisson event counts against the rate
integral, one-sample KS of the emitted xi against the exact CDF, independence of
the rate from dt (the carry), equality of the mean rate of methods I and II,
method I's saturation at W dt = 6, method III's factor 2, exact gyration in a
uniform B field, brute-force compaction.
"""
import math

import numpy as np

from . import philox, spectra, tables
from .constants import E_S, PAIR_GAMMA_MIN, PHOTON_XI_MIN_GAMMA, RATE_UNIT

DEAD_ID = np.uint64(0xFFFFFFFFFFFFFFFF)
KMAX = 4


# ------------------------------------------------------------------- fields
def standing_wave(x, t, a0):
    """Two counter-propagating circularly polarised waves (k = omega = 1):
    E = a0 cos x (0, cos t, sin t),  B = a0 sin x (0, cos t, sin t).
    An exact vacuum solution of Maxwell's equations in normalised units."""
    x = np.asarray(x, dtype=np.float64)
    cx, sx = np.cos(x), np.sin(x)
    ct, st = math.cos(t), math.sin(t)
    z = np.zeros_like(x)
    E = np.stack([z, a0 * cx * ct, a0 * cx * st], axis=-1)
    B = np.stack([z, a0 * sx * ct, a0 * sx * st], axis=-1)
    return E, B


def standing_wave_grid(n, L, a0, t):
    """Node values on an n^3 collocated periodic grid of side L, as arrays
    E[c, ix, iy, iz] and B[c, ix, iy, iz]."""
    xs = np.arange(n) * (L / n)
    E1, B1 = standing_wave(xs, t, a0)           # (n, 3)
    E = np.broadcast_to(E1.T[:, :, None, None], (3, n, n, n)).copy()
    B = np.broadcast_to(B1.T[:, :, None, None], (3, n, n, n)).copy()
    return E, B


def gather_tsc(Eg, Bg, L, x):
    """Quadratic-spline (TSC) interpolation on a periodic collocated grid:
    nearest node j = floor(x/dx + 1/2), d = x/dx - j, weights
    (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2) on nodes j-1, j, j+1."""
    n = Eg.shape[1]
    dx = L / n
    g = np.asarray(x, dtype=np.float64) / dx
    j = np.floor(g + 0.5)
    d = g - j
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=-1)  # (N,3,3)
    j = j.astype(np.int64)
    E = np.zeros(x.shape, dtype=np.float64)
    B = np.zeros(x.shape, dtype=np.float64)
    for a in range(3):
        ia = (j[:, 0] + a - 1) % n
        for b in range(3):
            ib = (j[:, 1] + b - 1) % n
            for c in range(3):
                ic = (j[:, 2] + c - 1) % n
                wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                E += wt[:, None] * Eg[:, ia, ib, ic].T
                B += wt[:, None] * Bg[:, ia, ib, ic].T
    return E, B


# --------------------------------------------------------------------- push
def boris(p, E, B, q, dt):
    """Relativistic Boris rotation; p in m_e c, q in units of e."""
    pm = p + 0.5 * q * dt * E
    g = np.sqrt(1.0 + np.sum(pm * pm, axis=-1))
    t = (0.5 * q * dt / g)[:, None] * B
    pp = pm + np.cross(pm, t)
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=-1))[:, None]
    return pm + np.cross(pp, s) + 0.5 * q * dt * E


def wrap(x, L):
    return x if L is None else np.mod(x, L)


def init_tau(ids, seed, step=0):
    """Initial optical depth tau = -ln u from purpose INIT_TAU, k = 0."""
    r = philox.stream(ids, seed, step, philox.INIT_TAU, 0)
    return -np.log(philox.uniform(r[..., 0]))


# ------------------------------------------------------------------ leptons
class RadSampler:
    """Rate and inverse CDF as the kernel sees them: float64 master values
    (double-precision species) or the 16-bit LDS copy and float32 ln h
    (single-precision species)."""

    def __init__(self, tab: tables.RadTable, storage="f64"):
        self.tab = tab
        self.t = tab.t
        if storage == "f64":
            self.S = tab.s
            self.ln_h = tab.ln_h
        elif storage == "q16":
            s0, sc, q = tables.quantize_rows(tab.s)
            self.S = tables.dequantize_rows(s0, sc, q)
            self.ln_h = tab.ln_h.astype(np.float32).astype(np.float64)
        else:
            raise ValueError(storage)
        self._tab_view = tables.RadTable(tab.kind, tab.chi, self.ln_h, tab.t, self.S, tab.chi_max)

    def rate(self, chi, gamma):
        return tables.rate_rad(self._tab_view, chi, gamma)

    def sample(self, chi, u_xi, u_row):
        return tables.sample_rad(self.S, self.t, chi, u_xi, u_row, self.tab.chi_max)


def lepton_step(x, p, tau, ids, E, B, *, q, dt, step, seed, sampler, next_id,
                L=None, kmax=KMAX, recoil=True):
    """One step for a lepton species.  Returns a dict with the new state,
    the appended photons (ordered by parent index, event k), the indices
    of particles with at least one event ('emitters'), and counters."""
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    tau = np.array(tau, dtype=np.float64)
    ids = np.asarray(ids, dtype=np.uint64)
    N = x.shape[0]

    p = boris(p, E, B, q, dt)
    gam = np.sqrt(1.0 + np.sum(p * p, axis=-1))
    x = wrap(x + p / gam[:, None] * dt, L)
    pabs0 = np.sqrt(np.sum(p * p, axis=-1))
    nhat = p / np.where(pabs0 > 0, pabs0, 1.0)[:, None]   # direction kept by recoil
    chi = spectra.chi_lepton(p, E, B)
    W = sampler.rate(chi, gam)
    rem = np.full(N, dt)
    active = (W > 0) & (tau <= W * rem)
    emitters = np.nonzero(active)[0]

    recs = []   # (parent, k, gamma_ph, tau_ph)
    n_events = 0
    n_reject = 0
    for k in range(kmax):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        n_events += idx.size
        rem[idx] -= tau[idx] / W[idx]
        r = philox.stream(ids[idx], seed, step, philox.LEPTON_EVENT, k)
        u = philox.uniform(r)
        xi, om = sampler.sample(chi[idx], u[:, 0], u[:, 2])
        gph = xi * gam[idx]
        acc = gph >= PHOTON_XI_MIN_GAMMA
        n_reject += int(np.count_nonzero(~acc))
        a = idx[acc]
        for par, g_ph, t_ph in zip(a, gph[acc], -np.log(u[acc, 3])):
            recs.append((int(par), k, float(g_ph), float(t_ph)))
        if recoil:   # recoil along the momentum direction
            gnew = np.maximum(om[acc] * gam[a], 1.0)
            pnew = np.sqrt(np.maximum(gnew * gnew - 1.0, 0.0))
            p[a] = nhat[a] * pnew[:, None]
            gam[a] = gnew
            chi[a] = spectra.chi_lepton(p[a], E[a], B[a])
            W[a] = sampler.rate(chi[a], gam[a])
        tau[idx] = -np.log(u[:, 1])
        still = (W[idx] > 0) & (tau[idx] <= W[idx] * rem[idx])
        active[:] = False
        active[idx[still]] = True
    n_capped = int(np.count_nonzero(active))
    tau = tau - W * rem

    recs.sort(key=lambda r: (r[0], r[1]))
    nph = len(recs)
    par = np.array([r[0] for r in recs], dtype=np.int64)
    gph = np.array([r[2] for r in recs], dtype=np.float64)
    # photon direction = lepton direction after the push (recoil keeps it)
    pdir = nhat[par] if nph else np.zeros((0, 3))
    photons = dict(
        x=x[par] if nph else np.zeros((0, 3)),
        k=pdir * gph[:, None] if nph else np.zeros((0, 3)),
        tau=np.array([r[3] for r in recs], dtype=np.float64),
        id=(np.uint64(next_id) + np.arange(nph, dtype=np.uint64)),
        parent=par, event=np.array([r[1] for r in recs], dtype=np.int64),
        gamma=gph,
    )
    return dict(x=x, p=p, tau=tau, id=ids, chi=chi, W=W, photons=photons,
                emitters=emitters, n_events=n_events, n_reject=n_reject,
                n_capped=n_capped, next_id=int(next_id) + nph)


def lepton_step_method1_full(x, p, ids, E, B, *, q, dt, step, seed, sampler, next_id, L=None,
                             kmax=KMAX, recoil=True, substep=True, w_max=0.2, nmax=1024):
    """The paper's adopted generator (method I, text after Eq. 7, with the
    adaptive step of its Fig. 3 discussion): the step is split into
    N = ceil(W Dt / 0.2) sub-steps (N = 1 without sub-stepping); in sub-step j
    an event happens if W Dt / N > r_1, at most one per sub-step, with W
    recomputed after a recoil.  Sub-step j uses counter k = j of the particle's
    LEPTON_EVENT stream: outputs (u_xi, r_1, u_row, u_ph).  At most kmax events
    per step.  N is fixed by the rate at the start of the step."""
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    ids = np.asarray(ids, dtype=np.uint64)
    n = x.shape[0]
    p = boris(p, E, B, q, dt)
    gam = np.sqrt(1.0 + np.sum(p * p, axis=-1))
    x = wrap(x + p / gam[:, None] * dt, L)
    pabs0 = np.sqrt(np.sum(p * p, axis=-1))
    nhat = p / np.where(pabs0 > 0, pabs0, 1.0)[:, None]
    chi = spectra.chi_lepton(p, E, B)
    W = sampler.rate(chi, gam)
    N = np.ones(n, dtype=np.int64)
    if substep:
        N = np.where(W > 0, np.maximum(1, np.ceil(W * dt / w_max)), 1).astype(np.int64)
        N = np.minimum(N, nmax)
    j = np.zeros(n, dtype=np.int64)
    nev = np.zeros(n, dtype=np.int64)
    active = W > 0
    recs = []
    emitters = None
    n_capped = 0
    while np.any(active):
        idx = np.nonzero(active)[0]
        r = philox.stream(ids[idx], seed, step, philox.LEPTON_EVENT, j[idx].astype(np.uint32))
        u = philox.uniform(r)
        fire = W[idx] * dt / N[idx] > u[:, 1]
        f = idx[fire]
        if f.size:
            uf = u[fire]
            xi, om = sampler.sample(chi[f], uf[:, 0], uf[:, 2])
            gph = xi * gam[f]
            acc = gph >= PHOTON_XI_MIN_GAMMA
            for par, k_ev, g_ph, t_ph in zip(f[acc], nev[f][acc], gph[acc], -np.log(uf[acc, 3])):
                recs.append((int(par), int(k_ev), float(g_ph), float(t_ph)))
            a = f[acc]
            if recoil and a.size:
                gnew = np.maximum(om[acc] * gam[a], 1.0)
                pnew = np.sqrt(np.maximum(gnew * gnew - 1.0, 0.0))
                p[a] = nhat[a] * pnew[:, None]
                gam[a] = gnew
                chi[a] = spectra.chi_lepton(p[a], E[a], B[a])
                W[a] = sampler.rate(chi[a], gam[a])
            nev[f] += 1
        j[idx] += 1
        capped = (nev >= kmax) & (j < N) & active
        n_capped += int(np.count_nonzero(capped))
        active = active & (j < N) & (nev < kmax) & (W > 0)
    recs.sort(key=lambda r: (r[0], r[1]))
    nph = len(recs)
    par = np.array([r[0] for r in recs], dtype=np.int64)
    gph = np.array([r[2] for r in recs], dtype=np.float64)
    photons = dict(
        x=x[par] if nph else np.zeros((0, 3)),
        k=nhat[par] * gph[:, None] if nph else np.zeros((0, 3)),
        tau=np.array([r[3] for r in recs], dtype=np.float64),
        id=(np.uint64(next_id) + np.arange(nph, dtype=np.uint64)),
        parent=par, gamma=gph)
    return dict(x=x, p=p, id=ids, chi=chi, N=N, photons=photons, n_events=int(nev.sum()),
                n_capped=n_capped, next_id=int(next_id) + nph)


def lepton_step_method1(p, tau_unused, ids, E, B, *, q, dt, step, seed, sampler):
    """Method I of the paper: emit (at most once per step) if W dt > r_1.
    Only the decision is modelled (no push, no recoil), for the time-step
    study; r_1 = u_tau of event slot 0."""
    gam = np.sqrt(1.0 + np.sum(p * p, axis=-1))
    chi = spectra.chi_lepton(p, E, B)
    W = sampler.rate(chi, gam)
    r = philox.stream(ids, seed, step, philox.LEPTON_EVENT, 0)
    u = philox.uniform(r)
    return W * dt > u[:, 1]


# ------------------------------------------------------------------ photons
class PairSampler:
    def __init__(self, tab: tables.PairTable, storage="f64"):
        self.tab = tab
        self.t = tab.t
        if storage == "f64":
            self.S = tab.s
            self.L = tab.L
        elif storage == "q16":
            s0, sc, q = tables.quantize_rows(tab.s)
            self.S = tables.dequantize_rows(s0, sc, q)
            self.L = tab.L.astype(np.float32).astype(np.float64)
        else:
            raise ValueError(storage)
        self._tab_view = tables.PairTable(tab.chi_rate, self.L, tab.chi_cdf, tab.t, self.S, tab.chi_max)

    def rate(self, chi, gamma_ph):
        return tables.rate_pair(self._tab_view, chi, gamma_ph)

    def sample_half(self, chi, u_xi, u_row):
        return tables.sample_pair_half(self.S, self.t, chi, u_xi, u_row, self.tab.chi_max)


def photon_step(x, k, tau, ids, E, B, *, dt, step, seed, sampler, next_id,
                move=True, L=None):
    x = np.array(x, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    tau = np.array(tau, dtype=np.float64)
    ids = np.array(ids, dtype=np.uint64)
    alive = ids != DEAD_ID            # photons converted earlier are left as they are
    gph = np.sqrt(np.sum(k * k, axis=-1))
    khat = k / np.where(gph > 0, gph, 1.0)[:, None]
    if move:
        x = np.where(alive[:, None], wrap(x + khat * dt, L), x)
    chi = spectra.chi_photon(k, E, B)
    W = np.where(alive, sampler.rate(chi, gph), 0.0)
    ev = alive & (W > 0) & (tau <= W * dt)
    tau = np.where(ev | ~alive, tau, tau - W * dt)
    idx = np.nonzero(ev)[0]
    r = philox.stream(ids[idx], seed, step, philox.PHOTON_EVENT, 0)
    u = philox.uniform(r)
    flip = (r[:, 1] & np.uint32(1)).astype(bool)
    xh, omh = sampler.sample_half(chi[idx], u[:, 0], u[:, 1])
    xi_e = np.where(flip, omh, xh)
    xi_p = np.where(flip, xh, omh)
    ge = xi_e * gph[idx]
    gp = xi_p * gph[idx]
    pe = khat[idx] * np.sqrt(np.maximum(ge * ge - 1.0, 0.0))[:, None]
    pp = khat[idx] * np.sqrt(np.maximum(gp * gp - 1.0, 0.0))[:, None]
    npair = idx.size
    rank = np.arange(npair, dtype=np.uint64)
    electrons = dict(x=x[idx], p=pe, tau=-np.log(u[:, 2]),
                     id=np.uint64(next_id) + 2 * rank, xi=xi_e)
    positrons = dict(x=x[idx], p=pp, tau=-np.log(u[:, 3]),
                     id=np.uint64(next_id) + 2 * rank + np.uint64(1), xi=xi_p)
    ids[idx] = DEAD_ID
    return dict(x=x, k=k, tau=tau, id=ids, chi=chi, W=W, pairs=idx,
                electrons=electrons, positrons=positrons,
                next_id=int(next_id) + 2 * npair)


# --------------------------------------------------------------- compaction
def compact(ids, *arrays):
    """Stable removal of dead particles: destination = exclusive prefix sum
    of the alive flags."""
    alive = np.asarray(ids, dtype=np.uint64) != DEAD_ID
    dest = np.cumsum(alive) - alive
    n = int(alive.sum())
    outs = []
    for a in (ids,) + arrays:
        o = np.empty((n,) + np.asarray(a).shape[1:], dtype=np.asarray(a).dtype)
        o[dest[alive]] = np.asarray(a)[alive]
        outs.append(o)
    return outs


# --------------------------------------------------------------- retirement
# A photon can only convert while its optical depth tau is consumed at the pair
# rate W = RATE_UNIT h_pair(chi_ph) / gamma_ph (Eq. 6 and the generator after
# Eq. 7), and chi_ph = gamma_ph / E_S |k x (E + k x B)| <= gamma_ph F / E_S when F
# bounds |E| + |B| (Eq. 3).  With an envelope h_env >= h_pair that grows with chi,
# W_max = RATE_UNIT h_env(gamma_ph F / E_S) / gamma_ph bounds W, and a photon with
# tau >= W_max (t_end - t) cannot convert before t_end: it is retired, i.e.
# counted into a histogram of ln gamma_ph (the tally) and no longer followed.
# Envelope: h_env = 1.002 C chi exp(-8 / (3 chi)) (1 + chi / 4)^(-1/3) with
# Erber's C = 3 sqrt3 / (16 sqrt2), 0 below chi = 1e-2 (where the pair rate is
# taken as 0); it lies above the tabulated rate (pinned in test_oracle_pins).
TALLY_BINS = 65536
TALLY_LN_LO, TALLY_LN_HI = math.log(2.0), math.log(1e7)
ERBER_C = 3.0 * math.sqrt(3.0) / (16.0 * math.sqrt(2.0))


def h_pair_envelope(chi):
    chi = np.asarray(chi, dtype=np.float64)
    out = np.zeros_like(chi)
    ok = chi >= tables.PAIR_CHI_MIN
    c = chi[ok]
    out[ok] = 1.002 * ERBER_C * c * np.exp(-8.0 / (3.0 * c)) * (1.0 + 0.25 * c) ** (-1.0 / 3.0)
    return out


def pair_rate_max(gamma_ph, field_bound):
    g = np.asarray(gamma_ph, dtype=np.float64)
    w = RATE_UNIT * h_pair_envelope(g * field_bound / E_S) / np.where(g > 0, g, 1.0)
    return np.where(g >= PAIR_GAMMA_MIN, w, 0.0)


def retirable(tau, gamma_ph, field_bound, t_left):
    return np.asarray(tau) >= pair_rate_max(gamma_ph, field_bound) * t_left


def tally_add(counts, gamma_ph):
    """bin = floor((ln gamma - ln 2) / ((ln 1e7 - ln 2) / TALLY_BINS)), clamped."""
    b = np.floor((np.log(np.asarray(gamma_ph, dtype=np.float64)) - TALLY_LN_LO)
                 * (TALLY_BINS / (TALLY_LN_HI - TALLY_LN_LO)))
    np.add.at(counts, np.clip(b, 0, TALLY_BINS - 1).astype(np.int64), 1)


# ------------------------------------------------------------------ cascade
def cascade_step(st, *, Eg=None, Bg=None, L=None, dt, step, seed, rad, pair, kmax=KMAX,
                 E0=None, B0=None, retire=None):
    """One step of the emission and pair cascade, in the order the GPU runs it:
    photons present at the start move, see the field at their new position and
    may convert (pairs appended to both lepton species); then electrons (q = -1)
    and positrons (q = +1) are pushed and emit (photons appended); finally the
    converted photons are removed.  st: dict with species 'el', 'po', 'ph' (x, p,
    tau, id) and 'next_id'; updated in place.  Fields: the periodic grid Eg, Bg
    of side L, or (Eg None) the uniform E0, B0 in unbounded space.  retire =
    (t_end, F): photons that can no longer convert before t_end (see above) are
    counted into st['tally'] and dropped, new ones before they are appended (their
    ids are assigned all the same), the others after the pair pass."""
    if Eg is None:
        E0, B0 = np.asarray(E0, np.float64), np.asarray(B0, np.float64)

        def fields(x):
            return np.broadcast_to(E0, x.shape).copy(), np.broadcast_to(B0, x.shape).copy()
        L = None
    else:
        def fields(x):
            return gather_tsc(Eg, Bg, L, x)
    ph = st["ph"]
    if retire is not None:
        st.setdefault("tally", np.zeros(TALLY_BINS, dtype=np.int64))
        t_left = retire[0] - (step + 1) * dt
    if ph["id"].size:
        g = np.sqrt(np.sum(ph["p"] * ph["p"], axis=-1))
        kh = ph["p"] / np.where(g > 0, g, 1.0)[:, None]
        xm = wrap(ph["x"] + kh * dt, L)
        E, B = fields(xm)
        r = photon_step(xm, ph["p"], ph["tau"], ph["id"], E, B, dt=dt, step=step, seed=seed,
                        sampler=pair, next_id=st["next_id"], move=False)
        st["next_id"] = r["next_id"]
        ids = r["id"]
        if retire is not None:
            out = (ids != DEAD_ID) & retirable(r["tau"], g, retire[1], t_left)
            tally_add(st["tally"], g[out])
            ids = np.where(out, DEAD_ID, ids)
        ph.update(x=xm, tau=r["tau"], id=ids)
        for name, new in (("el", r["electrons"]), ("po", r["positrons"])):
            sp = st[name]
            for k in ("x", "p", "tau", "id"):
                sp[k] = np.concatenate([sp[k], new[k]])
    for name, q in (("el", -1.0), ("po", 1.0)):
        sp = st[name]
        if sp["id"].size == 0:
            continue
        E, B = fields(sp["x"])
        r = lepton_step(sp["x"], sp["p"], sp["tau"], sp["id"], E, B, q=q, dt=dt, step=step, seed=seed,
                        sampler=rad, next_id=st["next_id"], L=L, kmax=kmax)
        sp.update(x=r["x"], p=r["p"], tau=r["tau"])
        st["next_id"] = r["next_id"]
        new = r["photons"]
        keep = np.ones(new["id"].size, dtype=bool)
        if retire is not None:
            keep = ~retirable(new["tau"], new["gamma"], retire[1], t_left)
            tally_add(st["tally"], new["gamma"][~keep])
        for k, v in (("x", new["x"]), ("p", new["k"]), ("tau", new["tau"]), ("id", new["id"])):
            ph[k] = np.concatenate([ph[k], v[keep]])
    keep = ph["id"] != DEAD_ID
    for k in ("x", "p", "tau", "id"):
        ph[k] = ph[k][keep]
