"""Parity bars shared by the GPU tests: every pressure comparison against the
FP64 oracle is made per mode, both as a relative L2 norm and element by
element (the largest deviation at any query, relative to the largest
reference value of that mode), so that one wrong query or one lane of a
ragged tile cannot hide in a norm."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    """max_q |a_q - b_q| / max_q |b_q|"""
    a = np.asarray(a)
    b = np.asarray(b)
    if b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def mode_errors(got, ref):
    """(relative L2, element-wise max relative) per mode of [modes][points] arrays."""
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    return [(rel_l2(got[m], ref[m]), rel_max(got[m], ref[m])) for m in range(ref.shape[0])]


def check_modes(got, ref, tol, label="", quiet=False):
    """Assert both bars for every mode; print the per-mode errors first.
    Returns the list of (rel L2, element-wise) pairs."""
    errs = mode_errors(got, ref)
    if not quiet:
        say(f"  {label} per mode (rel L2 / element-wise): "
            + " ".join(f"{a:.1e}/{b:.1e}" for a, b in errs))
    bad = [(m, a, b) for m, (a, b) in enumerate(errs) if not (a <= tol and b <= tol)]
    assert not bad, f"{label}: modes over the {tol:g} bar: {bad}"
    return errs
