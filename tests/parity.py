"""Parity rules between the GPU search and the CPU oracle (shared by tests,
smoke check and benchmark).

Integer instances: bit-exact (same masks, same energies, same order).

Float32 instances (tolerance tau = 1e-5 * sum_{i<j} |J_ij|), with O the
oracle's set and T the oracle's S-th energy:
  (i)   every returned energy is within tau of the oracle energy of its mask;
  (ii)  every returned mask not in O has oracle energy <= T + 2 tau;
  (iii) every oracle mask not returned has oracle energy >= T - 2 tau;
  (iv)  the output is sorted by (returned energy, mask);
  (v)   masks are distinct and below 2^N.
"""

from __future__ import annotations

import numpy as np


def tau_of(J) -> float:
    return 1e-5 * float(np.abs(np.triu(np.asarray(J, dtype=np.float64), 1)).sum())


def sorted_by_key(masks, energies) -> bool:
    m = np.asarray(masks, dtype=np.uint64)
    e = np.asarray(energies)
    if len(m) < 2:
        return True
    o = np.lexsort((m, e))
    return bool(np.all(o == np.arange(len(m))))


def check_int(masks, energies, o_masks, o_energies, what=""):
    m = np.asarray(masks, dtype=np.uint64)
    e = np.asarray(energies, dtype=np.int64)
    assert len(m) == len(o_masks), (what, len(m), len(o_masks))
    bad = np.nonzero((m != o_masks) | (e != o_energies))[0]
    assert len(bad) == 0, "%s: first mismatch at %d: gpu (%d, %d) oracle (%d, %d)" % (
        what, bad[0], m[bad[0]], e[bad[0]], o_masks[bad[0]], o_energies[bad[0]])


def check_f32(N, J, masks, energies, o_masks, o_energies, oracle_energy, what=""):
    """oracle_energy(mask) -> float64 energy (the oracle's Eq. 1)."""
    tau = tau_of(J)
    m = np.asarray(masks, dtype=np.uint64)
    e = np.asarray(energies, dtype=np.float64)
    S = len(o_masks)
    assert len(m) == S, (what, len(m), S)
    assert len(set(m.tolist())) == S, what + ": duplicate masks"
    assert int(m.max()) < (1 << N), what + ": mask out of range"
    assert sorted_by_key(m, np.asarray(energies, dtype=np.float32)), what + ": not sorted"
    eo = np.array([oracle_energy(int(x)) for x in m])
    err = np.abs(eo - e)
    assert err.max() <= tau, "%s: energy error %.3g > tau %.3g" % (what, err.max(), tau)
    T = float(o_energies[-1])
    O = set(np.asarray(o_masks, dtype=np.uint64).tolist())
    G = set(m.tolist())
    for x, ex in zip(m.tolist(), eo):
        if x not in O:
            assert ex <= T + 2 * tau, "%s: extra mask %d at %.9g > T + 2tau (%.9g)" % (
                what, x, ex, T + 2 * tau)
    for x, ex in zip(np.asarray(o_masks, dtype=np.uint64).tolist(), o_energies):
        if x not in G:
            assert ex >= T - 2 * tau, "%s: missing mask %d at %.9g < T - 2tau (%.9g)" % (
                what, x, ex, T - 2 * tau)
    return err.max(), tau
