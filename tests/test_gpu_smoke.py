"""The smoke entry point (one 32x32 factorization + solve against the oracle)
must pass as it is run on its own."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def test_smoke_entry_point():
    import __graft_entry__
    __graft_entry__.smoke()
