"""The FP64 oracle against what the paper and the mathematics fix (CPU only).

Each pin is described in tests/oracle_pins.py.  The last test plants every
mutation of MUTATIONS in the oracle and checks that some pin fails, so that a
plausible mistake anywhere in the oracle (a dropped term, a wrong sign, index
or axis) cannot pass the battery unnoticed.
"""
import pytest

import oracle
import oracle_pins as P
from oracle import SCHEME_LIE


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle._load()


@pytest.mark.parametrize("name", sorted(P.ALL_PINS))
def test_pin(name):
    ok, detail = P.ALL_PINS[name]()
    assert ok, f"{name}: {detail}"


def test_pin_paper_first_order_formula():
    """The printed product formula (V first, coefficients at t_j = j s;
    App. C.2.1 eq. prod_qhd, App. E.1 Algorithm 1) is first order."""
    ok, detail = P.pin_time_order(scheme=SCHEME_LIE)
    assert ok, detail


@pytest.mark.parametrize("pin", [P.pin_yoshida_one_step, P.pin_yoshida_order, P.pin_yoshida_reversal])
def test_pin_fourth_order_composition(pin):
    ok, detail = pin()
    assert ok, detail


def test_fourth_order_pins_catch_a_wrong_weight(monkeypatch):
    """A plausible mistake in the composition (w0 = 1 - w1, i.e. stages that do not
    sum to dt) planted in the pins' own weights makes the one-step pin fail."""
    monkeypatch.setattr(P, "yoshida_weights", lambda: (1.0 / (2.0 - 2.0 ** (1.0 / 3.0)),
                                                      1.0 - 1.0 / (2.0 - 2.0 ** (1.0 / 3.0)),
                                                      1.0 / (2.0 - 2.0 ** (1.0 / 3.0))))
    ok, _ = P.pin_yoshida_one_step()
    assert not ok


@pytest.mark.parametrize("mutation", sorted(oracle.MUTATIONS))
def test_planted_mistake_is_caught(mutation):
    code = oracle.MUTATIONS[mutation]
    for name, fn in P.ALL_PINS.items():
        ok, _ = fn(mutation=code)
        if not ok:
            return
    pytest.fail(f"no pin catches the planted mistake {mutation!r}")
