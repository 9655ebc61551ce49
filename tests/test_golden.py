"""The oracle still reproduces its frozen regression values (tests/golden/oracle_values.json)."""
import json
import os

import numpy as np

from oracle import green, kernel, mie, ops
from paper_1910_13844_amd import workloads

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


def cz(v):
    return complex(v[0], v[1])


def test_ghat_values():
    d = G["ghat_t_n8"]
    got = green.ghat_t(np.array(d["s"]), d["k"], d["R"])
    ref = np.array([cz(v) for v in d["values"]])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_kernel_and_operator_values():
    k = workloads.k_of()
    gm = kernel.gm_coset(8, 4, k)
    d = G["gm_n8_p4"]
    for p, v in zip(d["points"], d["values"]):
        assert abs(gm[tuple(p)] - cz(v)) <= 1e-13 * max(1e-3, abs(cz(v)))
    v = workloads.random_field(11, (8, 8, 8))
    Gv = ops.G_fft(np.fft.fftn(gm), v)
    d = G["Gv_n8_p4_seed11"]
    for p, val in zip(d["points"], d["values"]):
        assert abs(Gv[tuple(p)] - cz(val)) <= 1e-12 * abs(cz(val))


def test_mie_coefficients():
    d = G["mie_sphere32"]
    A, B = mie.coefficients(d["k"], d["k1"], d["a"], len(d["A"]) - 1)
    assert np.allclose(A, [cz(v) for v in d["A"]], rtol=1e-12, atol=1e-15)
    assert np.allclose(B, [cz(v) for v in d["B"]], rtol=1e-12, atol=1e-15)
