"""Helpers for the GPU parity tests: error statistics against the oracle."""
import numpy as np


def rel(a, b):
    """Relative L2 error ||a - b|| / ||b||."""
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elementwise(got, ref, theta_axis, last_wave_from=None):
    """Element-wise error relative to the rms of the reference: max |got - ref| / rms(ref)
    over all samples, over the 4 theta rows next to each pole, and (when given) over the
    rows theta >= last_wave_from (the last wave of a 16-wave theta tile)."""
    d = np.abs(got - ref)
    rms = float(np.sqrt(np.mean(ref ** 2))) or 1e-300
    n = ref.shape[theta_axis]
    pole = np.concatenate([np.arange(min(4, n)), np.arange(max(n - 4, 0), n)])
    out = {"all": float(d.max()) / rms, "pole": float(np.take(d, pole, axis=theta_axis).max()) / rms}
    if last_wave_from is not None and last_wave_from < n:
        out["last_wave"] = float(np.take(d, np.arange(last_wave_from, n), axis=theta_axis).max()) / rms
    return out


def fmt(stats):
    return " ".join(f"{k}={v:.1e}" for k, v in stats.items())
