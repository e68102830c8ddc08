"""Philox4x32-10 counter-based generator and the stream convention
(test infrastructure only).

Philox4x32-10 follows Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; each of the
10 rounds multiplies counter words 0 and 2 by the constants 0xD2511F53 and
0xCD9E8D57, takes the 64-bit products' high and low halves, and permutes/xors
them with the other two counter words and the key; between rounds the key is
advanced by the Weyl constants 0x9E3779B9 and 0xBB67AE85.

Stream convention of the Monte Carlo step (shared by the GPU, written separately):
    key     = (id_lo, id_hi ^ seed)
    counter = (step_lo, (step_hi & 0x00FFFFFF) | purpose << 24, k, 0)
    purpose INIT_TAU = 0, LEPTON_EVENT = 1, PHOTON_EVENT = 2
A lepton's k-th event in a step uses outputs (u_xi, u_tau, u_row, u_tau_photon);
a photon's pair event uses k = 0 for (u_xi, u_row, u_tau_electron,
u_tau_positron) and the low bit of the raw u_row word (a bit the uniform
mapping below discards) for the electron/positron exchange.

Uniform mapping: u = ((x >> 9) + 0.5) * 2^-23, which lies in [2^-24, 1 - 2^-24] and
is exact in float32 and float64, so both sides see identical u.

Pinned by tests/test_oracle_pins.py: the Random123 known-answer vectors for
philox4x32_10 (zero counter/key, all-ones counter/key, and the pi-digits case).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

INIT_TAU, LEPTON_EVENT, PHOTON_EVENT = 0, 1, 2


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32; key: (..., 2) uint32 -> (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32).copy()
    k1 = np.asarray(key[..., 1], dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            p0 = c[0].astype(np.uint64) * M0
            p1 = c[2].astype(np.uint64) * M1
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniform(x):
    """u = ((x >> 9) + 0.5) * 2^-23 in float64 (exact)."""
    return ((np.asarray(x, dtype=np.uint32) >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def stream(ids, seed, step, purpose, k):
    """Raw 4 x uint32 outputs for particle ids (uint64 array) at (step, purpose, k)."""
    ids = np.asarray(ids, dtype=np.uint64)
    n = ids.shape
    key = np.empty(n + (2,), dtype=np.uint32)
    key[..., 0] = (ids & MASK32).astype(np.uint32)
    key[..., 1] = ((ids >> np.uint64(32)).astype(np.uint32)) ^ np.uint32(seed)
    ctr = np.empty(n + (4,), dtype=np.uint32)
    step = np.uint64(step)
    ctr[..., 0] = np.uint32(int(step) & 0xFFFFFFFF)
    ctr[..., 1] = np.uint32(((int(step) >> 32) & 0x00FFFFFF) | (int(purpose) << 24))
    ctr[..., 2] = np.asarray(k, dtype=np.uint32)
    ctr[..., 3] = np.uint32(0)
    return philox4x32_10(ctr, key)
