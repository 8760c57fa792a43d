"""Error behaviour of the oracle's verbs (CPU): the consistency checks that
the paper runs before a simulation (Sec. 2: referenced molecules exist,
probabilities and compartments are coherent) and capacity overflow."""
import pytest

import oracle
import workloads as W


def base(**kw):
    return W.Model("e", W.SPHERE, 1e-6, 0, [W.Species("A", 1.0, 10), W.Species("B", 1.0, 10)],
                   [], outer_radius_um=1.0, capacity=64, **kw)


@pytest.mark.parametrize("rule", [
    W.bimol(0, 5, 1, -1, 0.01, 0.5),                       # unknown species
    W.bimol(0, 1, 1, -1, 0.0, 0.5),                        # zero radius
    W.bimol(0, 1, 1, -1, 0.01, 1.5),                       # p > 1
    W.unimol(0, -1, 0.1, placement=W.SPLIT, p2=1),         # split without first product
    W.unimol(0, -1, 0.1, placement=W.TRANSLOCATE, release=0.005, from_comp=0, to_comp=1),
])
def test_invalid_rules_rejected(rule):
    m = base()
    m.rules = [rule]
    with pytest.raises(oracle.OracleError) as ei:
        oracle.OracleSim(m)
    assert ei.value.code == -1


def test_second_rule_for_a_pair_rejected():
    m = base()
    m.rules = [W.bimol(0, 1, 1, -1, 0.01, 0.5), W.bimol(1, 0, 0, -1, 0.01, 0.5)]
    with pytest.raises(oracle.OracleError):
        oracle.OracleSim(m)


def test_unimolecular_probabilities_above_one_rejected_at_finalize():
    m = base()
    m.rules = [W.unimol(0, -1, 0.6), W.unimol(0, 1, 0.6)]
    s = oracle.OracleSim(m)
    with pytest.raises(oracle.OracleError) as ei:
        s.step(1)
    assert ei.value.code == -1


def test_capacity_overflow_is_sticky():
    m = base()
    m.species = [W.Species("G", 0.0, 10), W.Species("M", 1.0, 0)]
    m.rules = [W.unimol(0, -1, 1.0, placement=W.EMIT, p2=1, release=0.005)]
    m.capacity = 25
    s = oracle.OracleSim(m)
    s.step(1)
    with pytest.raises(oracle.OracleError) as ei:
        s.step(1)
    assert ei.value.code == -4
    with pytest.raises(oracle.OracleError):
        s.step(1)


def test_bad_geometry_rejected():
    m = base()
    m.outer_radius_um = -1.0
    with pytest.raises(oracle.OracleError):
        oracle.OracleSim(m)
