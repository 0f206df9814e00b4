"""Shared test helpers: per-field relative errors and state conversion."""
import numpy as np

RATE_FIELDS = ("drho", "dvx", "dvy", "dvz", "dE")


def field_relerr(gpu: dict, ref: dict, fields=RATE_FIELDS) -> dict:
    """Per-field relative error max_i |f_gpu - f_ref| / max_i |f_ref|.

    The velocity-rate components share one denominator, the largest of the
    three component maxima, so a component that is ~0 everywhere is judged
    against the scale of the vector field.
    """
    out = {}
    vmax = max(np.abs(ref[k]).max() for k in ("dvx", "dvy", "dvz") if k in ref) \
        if any(k in ref for k in ("dvx", "dvy", "dvz")) else 0.0
    for k in fields:
        a = np.asarray(gpu[k], np.float64)
        b = np.asarray(ref[k], np.float64)
        den = vmax if k in ("dvx", "dvy", "dvz") else np.abs(b).max()
        den = den if den > 0 else 1.0
        out[k] = float(np.abs(a - b).max() / den) if a.size else 0.0
    return out


def to_np(t):
    return t.detach().cpu().numpy()


def rates_np(out: dict) -> dict:
    return {k: to_np(v) for k, v in out.items() if hasattr(v, "detach")}
