"""Error measures used by the parity tests.

The bar: per cell and component |a - b| / max(|b|, f rms_cells(b)) <= 1e-5,
with f = 1e-3 (FLOOR), raised per component only where the 32-bit storage of
the floe state alone (the oracle rerun with its state rounded to the stored
formats after every step, tests/storage.py) moves that component by more than
a fifth of the allowance f rms 1e-5 (storage_floors): an FP32-state
implementation rounds its own state the same way (and evaluates the current in
FP32 besides), so its deviation from the exact oracle cannot fall below that
of the stored rerun, and it is allowed five times it."""
import numpy as np


FLOOR = 1e-3          # relative-error floor, a fraction of the component's rms over cells
TOL = 1e-5            # relative per-cell bar on moments and continuum after 1 and 10 steps
STORAGE_MARGIN = 5.0  # the storage-only deviation may use at most 1 / 5 of the allowance


def rel_err(a, b, floor=FLOOR):
    """Per cell and component: |a - b| / max(|b|, floor * rms over cells of b).

    floor is a scalar or one value per component (column).  A relative error
    is meaningless where a moment crosses zero (a cell whose momentum or drag
    sum cancels between floes); the floor measures such cells against a
    fraction of the component's scale instead."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b, axis=0, keepdims=True))
    den = np.maximum(np.abs(b), np.asarray(floor, np.float64).reshape(1, -1) * rms if np.ndim(floor) else floor * rms)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b) / den


def storage_floors(b, stored, tol=TOL, floor=FLOOR, margin=STORAGE_MARGIN):
    """Per-component floor of rel_err for comparing against the exact oracle
    result b: FLOOR, or, where the oracle with its state stored in the GPU's
    formats (`stored`) deviates from b by D (largest over cells), the floor at
    which D is 1 / margin of the allowance: margin D / (tol rms)."""
    b = np.asarray(b, np.float64)
    stored = np.asarray(stored, np.float64)
    rms = np.sqrt(np.mean(b * b, axis=0))
    dev = np.max(np.abs(stored - b), axis=0) if b.shape[0] else np.zeros(b.shape[1])
    need = np.where(rms > 0, margin * dev / (tol * np.where(rms > 0, rms, 1.0)), 0.0)
    return np.maximum(floor, need)


def report(a, b, floors, names=None):
    """One line per component: largest error at the floors, the floor, and the
    largest absolute error in units of the component's rms."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    e = rel_err(a, b, floors)
    rms = np.sqrt(np.mean(b * b, axis=0))
    fl = np.broadcast_to(np.asarray(floors, np.float64), (b.shape[1],))
    out = []
    for c in range(b.shape[1]):
        nm = names[c] if names else str(c)
        d = np.max(np.abs(a[:, c] - b[:, c])) / rms[c] if rms[c] > 0 else 0.0
        out.append(f"{nm}: {e[:, c].max():.1e} (floor {fl[c]:.1e}, |err|/rms {d:.1e})")
    return "; ".join(out)
