"""Seeded synthetic inputs for the QED Monte Carlo step.

This module only draws initial particle states and field samples; it holds
none of the method's arithmetic (no rates, spectra, chi or sampling).  Both the
HIP path's tests/benchmark and the CPU oracle start from these arrays.

Workloads (normalised units: t in 1/omega_0, x in c/omega_0, p in m_e c,
fields in m_e c omega_0 / e):

uniform_b_ensembles  three sub-ensembles in a static uniform B = b0 z, E = 0, with
    (b0, gamma) = (200, 206), (2000, 206), (2000, 2060): the paper's Fig. 1
    parameters (chi_e ~ 0.1, 1, 10); momenta in the x-y plane with a uniform
    random gyrophase; x = 0.
standing_wave_electrons  electrons uniform in the periodic box [0, 2 pi)^3 with
    Gaussian momenta of spread 10 m_e c per component.
pair_photons  photon directions (isotropic unit vectors), E and B drawn uniformly
    in the ball |E|, |B| <= 2000, and a target chi_ph log-uniform in [1e-2, 1e2];
    the caller turns the target into the photon energy with its own evaluation
    of the photon's quantum parameter (this module computes none).
sampler_inputs  log10 chi uniform in [-3, 2] with gamma = 1000, for the
    standalone sampler.
single_electron_runs  the Fig. 5 cascade seed: nrun copies of one electron with
    gamma_0 = 2e5 moving along +x, meant for a static B along z (the field is the
    caller's).  Run r sits at z = r: with B along z and every momentum in the
    x-y plane, z never changes, so each particle's z names its run.
"""
import math

import numpy as np

FIG1_TRIPLES = ((200.0, 206.0), (2000.0, 206.0), (2000.0, 2060.0))
BOX_L = 2.0 * math.pi


def uniform_b_ensembles(n_per, seed=0, triples=FIG1_TRIPLES):
    rng = np.random.default_rng(seed)
    out = []
    base = 0
    for b0, gamma in triples:
        phi = rng.uniform(0.0, 2.0 * math.pi, n_per)
        pm = math.sqrt(gamma * gamma - 1.0)
        p = np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n_per)], axis=-1)
        out.append(dict(b0=b0, gamma=gamma, x=np.zeros((n_per, 3)), p=p,
                        id=np.arange(base, base + n_per, dtype=np.uint64)))
        base += n_per
    return out


def standing_wave_electrons(n, seed=1, p_spread=10.0, L=BOX_L):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (n, 3))
    p = rng.normal(0.0, p_spread, (n, 3))
    return dict(x=x, p=p, id=np.arange(n, dtype=np.uint64))


def _isotropic(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _in_ball(rng, n, r):
    d = _isotropic(rng, n)
    rad = r * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    return d * rad[:, None]


def pair_photons(n, seed=2, chi_lo=1e-2, chi_hi=1e2, fmax=2000.0):
    rng = np.random.default_rng(seed)
    khat = _isotropic(rng, n)
    E = _in_ball(rng, n, fmax)
    B = _in_ball(rng, n, fmax)
    chi = 10.0 ** rng.uniform(math.log10(chi_lo), math.log10(chi_hi), n)
    return dict(x=np.zeros((n, 3)), khat=khat, E=E, B=B, id=np.arange(n, dtype=np.uint64), chi_target=chi)


def sampler_inputs(n, seed=3, gamma=1000.0):
    rng = np.random.default_rng(seed)
    chi = 10.0 ** rng.uniform(-3.0, 2.0, n)
    return dict(chi=chi, gamma=np.full(n, gamma), id=np.arange(n, dtype=np.uint64))


def single_electron_runs(nrun, gamma0=2e5):
    x = np.zeros((nrun, 3))
    x[:, 2] = np.arange(nrun, dtype=np.float64)
    p = np.zeros((nrun, 3))
    p[:, 0] = math.sqrt(gamma0 * gamma0 - 1.0)
    return dict(x=x, p=p, id=np.arange(nrun, dtype=np.uint64))
