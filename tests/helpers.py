"""Shared test helpers: state comparison at the parity bar.

Bar: the sorted label sets are identical (bit-exact) and every amplitude
differs by at most 1e-12 in complex modulus.
"""
import hashlib

import numpy as np

AMP_TOL = 1e-12


def assert_same_state(gpu, ref, tol=AMP_TOL, what=""):
    glo, ghi, gamp = gpu
    rlo, rhi, ramp = ref
    assert len(glo) == len(rlo), f"{what}: nnz {len(glo)} != oracle {len(rlo)}"
    assert np.array_equal(glo, rlo) and np.array_equal(ghi, rhi), f"{what}: label sets differ"
    if len(gamp):
        err = float(np.max(np.abs(gamp - ramp)))
        assert err <= tol, f"{what}: max |amp diff| {err:.3e} > {tol}"


def keys_digest(lo, hi) -> str:
    return hashlib.sha256(np.ascontiguousarray(lo, "<u8").tobytes() + np.ascontiguousarray(hi, "<u8").tobytes()
                          ).hexdigest()


def _void_keys(lo, hi):
    kb = np.empty((len(lo), 2), ">u8")
    kb[:, 0] = hi
    kb[:, 1] = lo
    return kb.view("V16").ravel()


def lookup(lo, hi, qlo, qhi):
    """Indices of the (qlo, qhi) labels in (lo, hi) sorted ascending by
    (hi, lo); -1 where absent."""
    v = _void_keys(lo, hi)
    q = _void_keys(np.asarray(qlo, np.uint64), np.asarray(qhi, np.uint64))
    pos = np.searchsorted(v, q)
    pos_c = np.minimum(pos, max(len(v) - 1, 0))
    hit = (pos < len(v)) & (v[pos_c] == q) if len(v) else np.zeros(len(q), bool)
    return np.where(hit, pos_c, -1)


def sorted_unique(lo, hi) -> bool:
    """True if labels sorted by (hi, lo) have no repeats."""
    if len(lo) < 2:
        return True
    return not bool(np.any((lo[1:] == lo[:-1]) & (hi[1:] == hi[:-1])))
