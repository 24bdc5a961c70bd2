"""Error measures of the parity tests (host-side numpy; no method arithmetic).

rel_l2    sqrt(sum a_i |phi_i - ref_i|^2 / sum a_i |ref_i|^2) over the sampled
          targets (areas a_i, or 1), Euclidean norms for vector outputs: the
          error metric E of the paper's §10.2 normalised by the reference.
elem_max  the worst relative error of one target,
              max_i |phi_i - ref_i| / max(|ref_i|, rms(ref)),
          floored at the sample's RMS so that a target where the field
          crosses zero does not divide by ~0.  A norm gate can hide an error
          confined to a few targets (one target off by 1e-4 moves the rel L2 of
          6,144 targets by ~1e-6); this one cannot.
"""

import numpy as np


def _norms(x):
    x = np.asarray(x, dtype=np.float64)
    return np.abs(x) if x.ndim == 1 else np.sqrt(np.sum(x * x, axis=1))


def rel_l2(got, ref, area=None):
    d = _norms(np.asarray(got) - np.asarray(ref))
    r = _norms(ref)
    a = np.ones_like(r) if area is None else np.asarray(area, dtype=np.float64)
    return float(np.sqrt(np.sum(a * d * d) / np.sum(a * r * r)))


def elem_max(got, ref):
    d = _norms(np.asarray(got) - np.asarray(ref))
    r = _norms(ref)
    rms = float(np.sqrt(np.mean(r * r)))
    return float(np.max(d / np.maximum(r, rms)))
