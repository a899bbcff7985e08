"""Error measures used by the parity tests."""
import numpy as np


FLOOR = 2e-2


def rel_err(a, b, floor=FLOOR):
    """Per cell and component: |a - b| / max(|b|, floor * rms over cells of b).

    A relative error is meaningless where a moment crosses zero (a cell whose
    momentum or drag sum cancels between floes).  The HIP path stores the floe
    state in FP32 (unit roundoff 6e-8) and evaluates the ocean current in FP32
    (measured error 1-2e-7 of the current's magnitude), so a cell sum carries an
    error of about 2e-7 of the field's scale whatever its own value; measured
    against 1e-5, that sets the floor at 2e-7 / 1e-5 = 2e-2 of the field rms."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b, axis=0, keepdims=True))
    den = np.maximum(np.abs(b), floor * rms)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b) / den
