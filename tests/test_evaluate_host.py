"""Host-side pieces of the evaluation layer (no GPU)."""
import math

import pytest

torch = pytest.importorskip("torch")


def test_relative_change():
    from paper_1706_06972_amd.evaluate import relative_change
    a = torch.tensor([3.0, 4.0])
    assert relative_change(a, a) == 0.0
    assert abs(relative_change(a, torch.zeros(2)) - 1.0) < 1e-15
    assert abs(relative_change(a, torch.tensor([3.0, 3.0])) - 0.2) < 1e-15
    assert relative_change(torch.zeros(2), torch.zeros(2)) == 0.0
    assert math.isinf(relative_change(torch.zeros(2), a))
