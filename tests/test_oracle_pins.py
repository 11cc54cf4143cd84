"""The CPU oracle against the paper's stated values, closed forms, Floyd-Warshall
and brute-force path search (see pins.py for what each check pins)."""
import pytest

import pins


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_pin(check, oracle_lib):
    kwargs = {}
    if check is pins.check_layers_vs_bfs:
        kwargs = dict(n_cases=400)
    elif check is pins.check_walk_bruteforce:
        kwargs = dict(n_cases=200, hmax=8)
    elif check is pins.check_walk_invariants:
        kwargs = dict(n_cases=200)
    check(oracle_lib, **kwargs)
