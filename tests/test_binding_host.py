"""Buffer checks of the Python binding, on the host: a buffer of the wrong
element type or too small for the context is refused before the library is
called, and host tensors are refused as device pointers.  The context here is
a stand-in handle whose sizes are planted in the binding's size cache; every
call here fails in the binding, so the library never sees the handle."""
import ctypes as C
import os

import pytest

torch = pytest.importorskip("torch")

from paper_1805_04155_amd import _ep  # noqa: E402

SIZES = {"dim": 2, "n_p": 9, "n_q": 9, "n_str": 3, "n_sc": 4, "n_colours": 4, "n_nodes": 25,
         "n_elems": 4, "n_int": 36, "n_dof": 50, "nnz": 900, "nnz_blocks": 225}


@pytest.fixture()
def fake_ctx():
    if not os.path.exists(_ep.LIB_PATH):
        from paper_1805_04155_amd import build
        build.build()
    h = C.c_void_p(0x7E57)
    _ep._SIZES[h.value] = dict(SIZES)
    yield h
    _ep._SIZES.pop(h.value, None)


def test_wrong_element_type_is_refused(fake_ctx):
    with pytest.raises(TypeError, match="u"):
        _ep.ep_constitutive(fake_ctx, torch.zeros(50, dtype=torch.float32))
    with pytest.raises(TypeError, match="flag"):
        _ep.ep_constitutive(fake_ctx, None, flag=torch.zeros(36, dtype=torch.int32))
    with pytest.raises(TypeError, match="ip"):
        _ep.ep_get_plastic(fake_ctx, torch.zeros(36, dtype=torch.int64))


def test_too_small_buffer_is_refused(fake_ctx):
    with pytest.raises(ValueError, match="sig"):
        _ep.ep_constitutive(fake_ctx, None, sig=torch.zeros(4 * 36 - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="F"):
        _ep.ep_internal_force(fake_ctx, torch.zeros(49, dtype=torch.float64))
    with pytest.raises(ValueError, match="pos"):
        _ep.ep_get_position_map(fake_ctx, torch.zeros(4 * 18 * 18 - 1, dtype=torch.int32))


def test_host_tensor_is_not_a_device_pointer(fake_ctx):
    with pytest.raises(TypeError, match="CUDA"):
        _ep.ep_spmv(fake_ctx, torch.zeros(50, dtype=torch.float64),
                    torch.zeros(50, dtype=torch.float64))
