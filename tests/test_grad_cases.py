"""The device-gradient cases sit away from every jump of the gradient (CPU)."""
import pytest

from grad_cases import CASES, IDS, conditioning, inputs, well_conditioned


@pytest.mark.parametrize("case", CASES[:-1], ids=IDS[:-1])
def test_gradient_cases_are_well_conditioned(case):
    w, V = inputs(case)
    c = conditioning(w["params"], w["obstacles"], w["x0"], V, case["step"])
    c.pop("oracle")
    assert well_conditioned(c), c
    assert c["n_weighted"] >= 1
