"""The oracle against the stored 60-digit fixtures (tests/golden/tiny_exact.json)."""
import numpy as np
import pytest

from golden_data import load
from oracle import metrics, reference, variants

U = 2.0 ** -53
FIX = load()


@pytest.mark.parametrize("name", sorted(FIX))
def test_chol_eqr_against_golden(name):
    d = FIX[name]
    q, r = reference.chol_eqr(d["A"], d["Z"])
    kap = np.linalg.cond(d["R"])
    assert metrics.r_forward_error(r, d["R"]) <= 100 * d["m"] * d["n"] * U * kap
    assert np.all(np.diag(r) > 0)


@pytest.mark.parametrize("name", sorted(FIX))
def test_golden_is_a_factorisation(name):
    d = FIX[name]
    a, z, q, r = d["A"], d["Z"], d["Q"], d["R"]
    assert metrics.residual_f(z, q, r) < 1e-15
    assert metrics.orth_loss_dd(a, q) < 1e-14 * max(1.0, metrics.diagnostics(a, z, q, r)["a_q2"])


def test_cgs2_against_golden():
    d = FIX["random_m24_n6"]
    q, r = variants.cgs2(d["A"], d["Z"])
    assert metrics.r_forward_error(r, d["R"]) < 1e-12
