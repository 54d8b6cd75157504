"""Error measures shared by the GPU parity tests (relative to the oracle)."""
import math

import numpy as np


def rms_err(a, b, ref=None):
    """sqrt(sum |a - b|^2 / sum |ref|^2), ref = b by default."""
    ref = np.asarray(b) if ref is None else np.asarray(ref)
    return math.sqrt(((np.asarray(a) - np.asarray(b)) ** 2).sum() / max((ref ** 2).sum(), 1e-300))


def per_particle(a, b, rms=None):
    """Per-particle errors of forces a against b ([n][3]):
    (max_i |dF_i| / rms F, max_i |dF_i| / max(|F_i|, rms F), the argmax of the
    latter). The first is the measure the rms error hides (one particle on a
    wrong path); the second judges a particle whose force is far above the
    rms (a close pair) against its own force."""
    a, b = np.asarray(a), np.asarray(b)
    if rms is None:
        rms = math.sqrt((b ** 2).sum(axis=1).mean())
    d = np.linalg.norm(a - b, axis=1)
    own = np.maximum(np.linalg.norm(b, axis=1), rms)
    k = int(np.argmax(d / own))
    return float(d.max() / rms), float((d / own)[k]), k
