import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__
    __graft_entry__.smoke()
