"""The round-trip check that the build's smoke() entry point runs."""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_smoke_entry_point():
    import __graft_entry__

    __graft_entry__.smoke()
