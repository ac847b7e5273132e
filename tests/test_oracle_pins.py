"""The oracle against its pins (CPU only).  See tests/oracle_pins.py for what each pin fixes."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("check", P.ALL_BASIC, ids=lambda c: c.__name__)
def test_basic_pin(check):
    check()


def test_invariances(small_2d_workload, abc16_workload):
    P.check_invariances(small_2d_workload, abc16_workload)


def test_relabel(small_2d_workload):
    P.check_relabel(small_2d_workload)


def test_adjoint_fd_16cubed(abc16_workload):
    # the 16^3 ABC instance in float64, central differences with h = 1e-6
    P.check_adjoint_fd(abc16_workload)


def test_adjoint_identities(abc16_workload):
    P.check_adjoint_identities(abc16_workload)
