"""Total rates and inverse-CDF tables, built by quadrature in float64
(test infrastructure only).

What the tables hold follows the paper's Monte Carlo generator: the total rate
W = int dW/dxi (text after Eq. 7, photons from Eq. 1 or 4, pairs from Eq. 6) and
the photon energy fraction obtained by inverting the cumulative spectrum,
int_{xi_min}^{xi^0} dW/dxi = r_2 W (Eq. 7).  The layout is fixed so that the GPU
builder and this oracle produce the same numbers from their own quadrature:

Photon emission ("rad"), formula I or II
  chi nodes     256, log-spaced over [1e-3, 1e2]
  rate          ln h(chi_i), h = int_0^1 S dxi (uncut; the cut at xi_min = 2/gamma is
                applied by rejecting samples, which thins the Poisson process)
  fine grid     per row, M = 1024 intervals uniform in s = logit(xi) over
                [logit(1e-15 chi), ln(60 chi)]; the upper end is where
                d = 2 xi / (3 (1-xi) chi) = 40.  Each interval is integrated with
                3-point Gauss-Legendre; below the lower end the analytic infrared
                tail int_0^xi S = 3 Gamma(2/3) (3 chi)^(2/3) xi^(1/3) / (sqrt3 pi)
                (from K_{2/3}(d) ~ Gamma(2/3)/2 (2/d)^(2/3)) is added.
  inverse CDF   256 quantile nodes uniform in t = logit(u) over
                [logit(1e-4), logit(1 - 1e-7)]; node value = s(u) solved on the
                cubic Hermite interpolant of the fine CDF (exact slopes), by 52
                bisections of the interval.  Sampling below u = 1e-4 uses the
                infrared law xi ~ u^3; above the last node it clamps.

Breit-Wheeler pairs (Eq. 6, "+" sign)
  rate          512 chi_ph nodes log-spaced over [1e-2, 1e2], stored as
                ln h_pair(chi) + 8 / (3 chi) (the exp(-8/(3 chi)) factor removed so
                that linear interpolation is accurate)
  inverse CDF   256 chi_ph rows over [1e-2, 1e2] for the half-spectrum
                xi in (0, 1/2] (Eq. 6 is symmetric under xi <-> 1 - xi); fine grid
                M = 1024 in s over [logit(xi_lo), 0], xi_lo where d exceeds its
                value at xi = 1/2 by 45; 256 quantile nodes uniform in logit(u) over
                [logit(1e-6), logit(1 - 1e-6)], clamped outside.

Lookups (rate_rad, rate_pair, sample_rad, sample_pair) are written out below in
float64 in the same steps the kernels take; "quantize" mirrors the 16-bit
storage the single-precision kernels stage in LDS.

Pinned by tests/test_oracle_pins.py: h(chi) asymptotes (5 chi / (2 sqrt3) *
(1 - 8 sqrt3 chi / 15) and 14 Gamma(2/3) chi^(2/3) / (9 3^(1/3))), Erber's pair
asymptote, xi <-> 1-xi symmetry, CDF monotone with P(1) = 1, quantiles against an
independent scipy quad of the spectrum, and sampled-spectrum KS against the exact
CDF.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import spectra
from .constants import GAMMA_2_3, RATE_UNIT

# ------------------------------------------------------------------ layout
RAD_NCHI, RAD_CHI_MIN, RAD_CHI_MAX = 256, 1e-3, 1e2
RAD_M = 1024
RAD_XI_LO_OVER_CHI = 1e-15
RAD_D_HI = 40.0
RAD_NU = 256
RAD_U_LO, RAD_U_HI = 1e-4, 1.0 - 1e-7

PAIR_NRATE, PAIR_NCDF = 512, 256
PAIR_CHI_MIN, PAIR_CHI_MAX = 1e-2, 1e2
PAIR_M = 1024
PAIR_DD = 45.0
PAIR_NU = 256
PAIR_U_LO, PAIR_U_HI = 1e-6, 1.0 - 1e-6

# small-chi expansion of h(chi) used below the rad table range
H_SMALL_C1 = 5.0 / (2.0 * math.sqrt(3.0))
H_SMALL_C2 = 8.0 * math.sqrt(3.0) / 15.0

_GL3_X = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
_GL3_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


def logit(u):
    u = np.asarray(u, dtype=np.float64)
    return np.log(u) - np.log1p(-u)


def chi_nodes(n, lo, hi):
    return np.exp(math.log(lo) + np.arange(n) * ((math.log(hi) - math.log(lo)) / (n - 1)))


def t_nodes(n, u_lo, u_hi):
    t_lo, t_hi = float(logit(u_lo)), float(logit(u_hi))
    return t_lo + np.arange(n) * ((t_hi - t_lo) / (n - 1))


# ------------------------------------------------------------- fine rows
@dataclass
class FineRow:
    """Cumulative spectrum of one chi row on its fine logit grid."""
    s: np.ndarray        # M+1 nodes
    F: np.ndarray        # cumulative (unnormalised) at the nodes, F[0] = tail
    rho: np.ndarray      # density in s at the nodes, S(xi) xi (1-xi)
    total: float


def _density(kind, s, chi):
    xi = 1.0 / (1.0 + np.exp(-s))
    om = 1.0 / (1.0 + np.exp(s))
    if kind == "I":
        S = spectra.formula_I_logit(s, chi)
    elif kind == "II":
        S = spectra.formula_II_logit(s, chi)
    elif kind == "pair":
        S = spectra.pair_logit(s, chi)
    elif kind == "classical":
        S = spectra.classical(xi, chi)
    else:
        raise ValueError(kind)
    return S * xi * om


def rad_bounds(chi):
    xi_lo = RAD_XI_LO_OVER_CHI * chi
    return math.log(xi_lo) - math.log1p(-xi_lo), math.log(1.5 * RAD_D_HI * chi)


def pair_bounds(chi):
    q = 2.0 / (8.0 + 3.0 * chi * PAIR_DD)
    xi_lo = 2.0 * q / (1.0 + math.sqrt(1.0 - 4.0 * q))
    return math.log(xi_lo) - math.log1p(-xi_lo), 0.0


def rad_ir_tail(chi, xi_lo):
    """int_0^xi_lo S dxi from the small-argument form of K_{2/3} (Eq. 1 / Eq. 4)."""
    return spectra.INV_SQRT3_PI * 3.0 * GAMMA_2_3 * (3.0 * chi) ** (2.0 / 3.0) * xi_lo ** (1.0 / 3.0)


def fine_row(kind, chi, M, need_rho=True):
    if kind == "pair":
        s_lo, s_hi = pair_bounds(chi)
        tail = 0.0
    else:
        s_lo, s_hi = rad_bounds(chi)
        tail = rad_ir_tail(chi, RAD_XI_LO_OVER_CHI * chi)
    ds = (s_hi - s_lo) / M
    s = s_lo + np.arange(M + 1) * ds
    sg = (s[:-1, None] + ds * _GL3_X[None, :]).reshape(-1)
    g = _density(kind, sg, chi).reshape(M, 3)
    I = ds * (g @ _GL3_W)
    F = tail + np.concatenate([[0.0], np.cumsum(I)])
    rho = _density(kind, s, chi) if need_rho else None
    return FineRow(s=s, F=F, rho=rho, total=float(F[-1]))


def _hermite(tau, p0, p1, d0, d1, ds):
    t2, t3 = tau * tau, tau * tau * tau
    return ((2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + tau) * ds * d0
            + (-2 * t3 + 3 * t2) * p1 + (t3 - t2) * ds * d1)


def quantile(row: FineRow, u, ir_tail):
    """s(u) on the cubic Hermite interpolant of the normalised fine CDF."""
    P = row.F / row.total
    d = row.rho / row.total
    M = len(row.s) - 1
    ds = row.s[1] - row.s[0]
    if u <= P[0]:
        if not ir_tail:
            return float(row.s[0])
        xi_lo = 1.0 / (1.0 + math.exp(-row.s[0]))
        xi = xi_lo * (u / P[0]) ** 3
        return math.log(xi) - math.log1p(-xi)
    if u >= P[M]:
        return float(row.s[M])
    m = int(np.searchsorted(P, u, side="right")) - 1
    m = min(max(m, 0), M - 1)
    lo, hi = 0.0, 1.0
    for _ in range(52):
        mid = 0.5 * (lo + hi)
        if _hermite(mid, P[m], P[m + 1], d[m], d[m + 1], ds) < u:
            lo = mid
        else:
            hi = mid
    return float(row.s[m] + 0.5 * (lo + hi) * ds)


# ------------------------------------------------------------ table builds
@dataclass
class RadTable:
    kind: str
    chi: np.ndarray      # (256,)
    ln_h: np.ndarray     # (256,)
    t: np.ndarray        # (256,) quantile nodes in logit(u)
    s: np.ndarray        # (256, 256) logit(xi) at the quantile nodes
    chi_max: float = RAD_CHI_MAX   # upper end of the chi nodes


@dataclass
class PairTable:
    chi_rate: np.ndarray   # (512,)
    L: np.ndarray          # (512,) ln h_pair + 8/(3 chi)
    chi_cdf: np.ndarray    # (256,)
    t: np.ndarray          # (256,)
    s: np.ndarray          # (256, 256) logit(xi) of the half spectrum
    chi_max: float = PAIR_CHI_MAX  # upper end of both chi grids


def build_rad_table(kind="I", rows=None, chi_max=RAD_CHI_MAX):
    """Photon table for formula I ("I"), II ("II") or the classical limit
    ("classical", Eq. 5 restricted to xi < 1, whose small-xi tail is the same as
    Eq. 1's).  rows: optional subset.  chi_max: upper end of the chi nodes
    (1e2 by default; larger for chi_0 ~ 4e4 as in Fig. 5)."""
    chi = chi_nodes(RAD_NCHI, RAD_CHI_MIN, chi_max)
    t = t_nodes(RAD_NU, RAD_U_LO, RAD_U_HI)
    u = 1.0 / (1.0 + np.exp(-t))
    idx = range(RAD_NCHI) if rows is None else rows
    ln_h = np.full(RAD_NCHI, np.nan)
    s = np.full((RAD_NCHI, RAD_NU), np.nan)
    for i in idx:
        row = fine_row(kind, chi[i], RAD_M)
        ln_h[i] = math.log(row.total)
        s[i] = [quantile(row, uk, ir_tail=True) for uk in u]
    return RadTable(kind=kind, chi=chi, ln_h=ln_h, t=t, s=s, chi_max=chi_max)


def build_pair_table(rate_rows=None, cdf_rows=None, chi_max=PAIR_CHI_MAX):
    chi_r = chi_nodes(PAIR_NRATE, PAIR_CHI_MIN, chi_max)
    chi_c = chi_nodes(PAIR_NCDF, PAIR_CHI_MIN, chi_max)
    t = t_nodes(PAIR_NU, PAIR_U_LO, PAIR_U_HI)
    u = 1.0 / (1.0 + np.exp(-t))
    L = np.full(PAIR_NRATE, np.nan)
    for i in (range(PAIR_NRATE) if rate_rows is None else rate_rows):
        row = fine_row("pair", chi_r[i], PAIR_M, need_rho=False)
        L[i] = math.log(2.0 * row.total) + 8.0 / (3.0 * chi_r[i])
    s = np.full((PAIR_NCDF, PAIR_NU), np.nan)
    for i in (range(PAIR_NCDF) if cdf_rows is None else cdf_rows):
        row = fine_row("pair", chi_c[i], PAIR_M)
        s[i] = [quantile(row, uk, ir_tail=False) for uk in u]
    return PairTable(chi_rate=chi_r, L=L, chi_cdf=chi_c, t=t, s=s, chi_max=chi_max)


# ---------------------------------------------------------- 16-bit storage
def quantize_rows(s):
    """Per-row 16-bit code of logit(xi): s = s0 + q * scale with s0 and scale
    rounded to float32 (the storage the single-precision kernels stage in LDS)."""
    s0 = s[:, 0].astype(np.float32)
    scale = ((s[:, -1] - s[:, 0]) / 65535.0).astype(np.float32)
    q = np.rint((s - s[:, :1]) / ((s[:, -1] - s[:, 0]) / 65535.0)[:, None])
    q = np.clip(q, 0, 65535).astype(np.uint16)
    return s0, scale, q


def dequantize_rows(s0, scale, q):
    return s0.astype(np.float64)[:, None] + q.astype(np.float64) * scale.astype(np.float64)[:, None]


# ------------------------------------------------------------------ lookups
def _grid_pos(chi, n, lo, hi):
    x = (np.log(chi) - math.log(lo)) / ((math.log(hi) - math.log(lo)) / (n - 1))
    return x


def h_rad(tab: RadTable, chi):
    """h(chi) by linear interpolation of ln h in ln chi; small-chi expansion
    below the table, chi^(2/3) growth above it; 0 at chi = 0."""
    chi = np.asarray(chi, dtype=np.float64)
    out = np.zeros_like(chi)
    pos = chi > 0
    c = np.where(pos, chi, 1.0)
    hi = tab.chi_max
    x = _grid_pos(c, RAD_NCHI, RAD_CHI_MIN, hi)
    i = np.clip(np.floor(x), 0, RAD_NCHI - 2).astype(np.int64)
    f = x - i
    inside = np.exp((1.0 - f) * tab.ln_h[i] + f * tab.ln_h[i + 1])
    below = H_SMALL_C1 * c * (1.0 - H_SMALL_C2 * c)
    above = np.exp(tab.ln_h[-1]) * (c / hi) ** (2.0 / 3.0)
    h = np.where(c < RAD_CHI_MIN, below, np.where(c > hi, above, inside))
    out[pos] = h[pos]
    return out


def rate_rad(tab, chi, gamma):
    """W_rad = alpha E_S h(chi) / gamma  [1/omega_0], uncut."""
    return RATE_UNIT * h_rad(tab, chi) / np.asarray(gamma, dtype=np.float64)


def h_pair(tab: PairTable, chi):
    chi = np.asarray(chi, dtype=np.float64)
    c = np.where(chi > 0, chi, 1.0)
    hi = tab.chi_max
    x = _grid_pos(c, PAIR_NRATE, PAIR_CHI_MIN, hi)
    i = np.clip(np.floor(x), 0, PAIR_NRATE - 2).astype(np.int64)
    f = x - i
    inside = np.exp((1.0 - f) * tab.L[i] + f * tab.L[i + 1] - 8.0 / (3.0 * c))
    above = np.exp(tab.L[-1] - 8.0 / (3.0 * hi)) * (c / hi) ** (2.0 / 3.0)
    h = np.where(c > hi, above, inside)
    return np.where(chi < PAIR_CHI_MIN, 0.0, h)


def rate_pair(tab, chi, gamma_ph):
    """W_pair = alpha E_S h_pair(chi_ph) / gamma_ph, zero below 2 m_e c^2."""
    g = np.asarray(gamma_ph, dtype=np.float64)
    w = RATE_UNIT * h_pair(tab, chi) / np.where(g > 0, g, 1.0)
    return np.where(g < 2.0, 0.0, w)


def _row_pick(chi, u_row, n, lo, hi):
    """Row index: linear interpolation of the CDF in ln chi realised by picking
    row i+1 with probability equal to the fractional position."""
    x = _grid_pos(chi, n, lo, hi)
    i = np.clip(np.floor(x), 0, n - 2).astype(np.int64)
    f = x - i
    row = i + (u_row < f).astype(np.int64)
    row = np.where(x < 0, 0, np.where(x >= n - 1, n - 1, row))
    return row


def _interp_s(S, row, u, t_nodes_, tail_cube, u_lo):
    t = np.log(u) - np.log1p(-u)
    n = S.shape[1]
    t_lo, dt = t_nodes_[0], (t_nodes_[-1] - t_nodes_[0]) / (n - 1)
    y = (t - t_lo) / dt
    j = np.clip(np.floor(y), 0, n - 2).astype(np.int64)
    f = y - j
    s = (1.0 - f) * S[row, j] + f * S[row, j + 1]
    s = np.where(y >= n - 1, S[row, n - 1], s)
    if tail_cube:
        s0 = S[row, 0]
        xi0 = 1.0 / (1.0 + np.exp(-s0))
        xi = xi0 * (u / u_lo) ** 3
        s_tail = np.log(xi) - np.log1p(-xi)
        s = np.where(y < 0, s_tail, s)
    else:
        s = np.where(y < 0, S[row, 0], s)
    return s


def sample_rad(S, t_nodes_, chi, u_xi, u_row, chi_max=RAD_CHI_MAX):
    """xi and 1-xi from the photon inverse CDF S (256 x 256 logit values).
    Below the table's chi range the row-0 sample is scaled by chi / chi_min
    (the classical spectrum depends on xi / chi); above it, the last row."""
    chi = np.asarray(chi, dtype=np.float64)
    row = _row_pick(chi, u_row, RAD_NCHI, RAD_CHI_MIN, chi_max)
    s = _interp_s(S, row, np.asarray(u_xi, np.float64), t_nodes_, True, RAD_U_LO)
    xi = 1.0 / (1.0 + np.exp(-s))
    om = 1.0 / (1.0 + np.exp(s))
    below = chi < RAD_CHI_MIN
    scale = np.where(below, chi / RAD_CHI_MIN, 1.0)
    xi_b = xi * scale
    return np.where(below, xi_b, xi), np.where(below, 1.0 - xi_b, om)


def sample_pair_half(S, t_nodes_, chi, u_xi, u_row, chi_max=PAIR_CHI_MAX):
    """xi in (0, 1/2] from the half-spectrum inverse CDF (chi >= 1e-2)."""
    chi = np.asarray(chi, dtype=np.float64)
    row = _row_pick(chi, u_row, PAIR_NCDF, PAIR_CHI_MIN, chi_max)
    s = _interp_s(S, row, np.asarray(u_xi, np.float64), t_nodes_, False, PAIR_U_LO)
    return 1.0 / (1.0 + np.exp(-s)), 1.0 / (1.0 + np.exp(s))
