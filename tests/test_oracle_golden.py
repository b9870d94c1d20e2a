"""The oracle against the relations the paper prints (tests/golden/paper_relations.json)."""

import json
import os

import numpy as np
import pytest

from oracle import model, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_relations.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_prandtl_to_b(golden):
    for item in golden["prandtl_b"]:
        assert model.b_from_prandtl(item["Pr"]) == pytest.approx(item["b"], abs=1e-15)


def test_b_range_keeps_lambda_positive_definite(golden):
    # A physical pressure tensor P = rho T delta + sigma is positive
    # semidefinite, so the traceless stress of a 3-D gas has eigenvalues in
    # [-rho T, 2 rho T]. lambda = T delta + b sigma / rho stays semidefinite for
    # every such stress exactly when -1/2 <= b <= 1.
    lo, hi = golden["b_range"]["min"], golden["b_range"]["max"]
    T, rho = np.array([1.3]), np.array([0.7])
    extremes = [rho[0] * T[0] * np.diag([2.0, -1.0, -1.0]),
                rho[0] * T[0] * np.diag([-1.0, 0.5, 0.5])]
    for b in np.linspace(lo, hi, 7):
        for s in extremes:
            assert np.linalg.eigvalsh(model.es_tensor(T, s[None], rho, b)[0]).min() >= -1e-12
    assert np.linalg.eigvalsh(model.es_tensor(T, extremes[0][None], rho, lo - 0.01)[0]).min() < 0
    assert np.linalg.eigvalsh(model.es_tensor(T, extremes[1][None], rho, hi + 0.01)[0]).min() < 0


def test_heat_capacity_relation(golden):
    hc = golden["heat_capacity"]
    assert (hc["D"] + 2) / 2 == hc["Cp"]


def test_eleventh_order_rule(golden):
    q = golden["quadrature"]
    c, w = quadrature.hermite_rule_1d(q["points_1d"])
    assert 2 * q["points_1d"] - 1 == q["degree"]
    for k in range(q["degree"] + 1):
        ref = 0.0 if k % 2 else float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0
        assert abs(np.sum(w * c ** k) - ref) < 1e-12 * np.sum(w * np.abs(c) ** k)


def test_d2q37_meets_the_minimum_degree_for_n4(golden):
    eo = golden["expansion_order"]
    vs = quadrature.d2q37()
    assert vs.N == eo["N"] and vs.degree >= eo["min_degree"]
