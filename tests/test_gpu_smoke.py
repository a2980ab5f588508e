"""The smoke entry point (one small propose+accept run checked against the
oracle) stays runnable."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_smoke_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__ as g
    g.smoke()
