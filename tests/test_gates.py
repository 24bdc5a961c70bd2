"""The element-wise gate catches what a norm gate hides (CPU, oracle data).

A mistake planted in the oracle's own result -- one target of config 1's
6,144 off by 1e-4 of its value -- moves the relative L2 error by only ~1e-6,
inside the FP32-form norm gate of 2e-6, while the worst per-target error
(floored at the RMS) reports it at full size.
"""

import numpy as np

from gates import rel_l2, elem_max
from oracle import direct
from workloads import cubed_sphere_grid, real_y43


def test_single_target_error_passes_norm_gate_fails_elementwise():
    P, A = cubed_sphere_grid(32)
    ref = direct(1, P, P, real_y43(P) * A)
    r = np.abs(ref)
    k = int(np.argmin(np.abs(r - np.sqrt(np.mean(r * r)))))  # a target of typical size
    bad = ref.copy()
    bad[k] *= 1.0 + 1e-4
    assert rel_l2(bad, ref, A) < 2e-6            # hidden by the norm gate
    assert 0.9e-4 < elem_max(bad, ref) < 1.1e-4  # seen element-wise


def test_elem_max_floors_at_rms_and_uses_vector_norms():
    ref = np.array([1.0, -1.0, 1e-12, 1.0])
    got = ref + np.array([0.0, 0.0, 1e-6, 0.0])
    # a tiny reference value does not blow the measure up: floor at the RMS
    assert abs(elem_max(got, ref) - 1e-6 / np.sqrt(np.mean(ref * ref))) < 1e-15
    v = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 5.0]])
    w = v + np.array([[0.0, 0.0, 0.05], [0.0, 0.0, 0.0]])
    assert abs(elem_max(w, v) - 0.01) < 1e-15
    assert abs(rel_l2(w, v) - 0.05 / np.sqrt(50.0)) < 1e-15
