"""Host-side checks of the torch binding: a checkpoint store or gradient
buffer that does not match what the library will write or read through the
pointer is refused with ValueError/TypeError before any library call.

The shape/dtype/device/layout rules are checked on CPU tensors here (no GPU
needed); tests/test_binding_checks_gpu.py drives the same rules through
api.run and api.adjoint_run on the device."""
import pytest
import torch

from paper_2107_00555_amd import api


def _state(shape=(6, 5, 4), dtype=torch.float64):
    return torch.zeros(shape, dtype=dtype)


@pytest.mark.parametrize("T,k,slots", [(10, 3, 4), (10, 5, 2), (1, 7, 1), (9, 1, 9), (0, 4, 0)])
def test_checkpoint_store_of_the_right_shape_is_accepted(T, k, slots):
    u = _state()
    ck = torch.zeros((slots,) + tuple(u.shape), dtype=u.dtype)
    assert api.check_ckpt(ck, T, k, u) is ck
    assert api.num_slots(T, k) == slots


def test_checkpoint_store_with_too_few_slots_is_refused():
    u = _state()
    with pytest.raises(ValueError, match="shaped"):
        api.check_ckpt(torch.zeros((3,) + tuple(u.shape), dtype=u.dtype), 10, 3, u)


def test_checkpoint_store_with_too_many_slots_is_refused():
    u = _state()
    with pytest.raises(ValueError, match="shaped"):
        api.check_ckpt(torch.zeros((5,) + tuple(u.shape), dtype=u.dtype), 10, 3, u)


def test_checkpoint_store_of_another_field_shape_is_refused():
    u = _state()
    with pytest.raises(ValueError, match="shaped"):
        api.check_ckpt(torch.zeros((4, 6, 5, 5), dtype=u.dtype), 10, 3, u)
    with pytest.raises(ValueError, match="shaped"):
        api.check_ckpt(torch.zeros((4 * 6, 5, 4), dtype=u.dtype), 10, 3, u)


def test_checkpoint_store_of_another_dtype_is_refused():
    u = _state()
    with pytest.raises(ValueError, match="dtype"):
        api.check_ckpt(torch.zeros((4,) + tuple(u.shape), dtype=torch.float32), 10, 3, u)
    u32 = _state(dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        api.check_ckpt(torch.zeros((4,) + tuple(u32.shape), dtype=torch.float64), 10, 3, u32)


def test_checkpoint_store_on_another_device_is_refused():
    u = _state().to("meta")
    with pytest.raises(ValueError, match="device"):
        api.check_ckpt(torch.zeros((4,) + tuple(u.shape), dtype=u.dtype), 10, 3, u)


def test_non_contiguous_checkpoint_store_is_refused():
    u = _state()
    ck = torch.zeros((4,) + tuple(reversed(u.shape)), dtype=u.dtype).permute(0, 3, 2, 1)
    assert tuple(ck.shape) == (4,) + tuple(u.shape)
    with pytest.raises(ValueError, match="contiguous"):
        api.check_ckpt(ck, 10, 3, u)


def test_checkpoint_interval_below_one_is_refused():
    u = _state()
    with pytest.raises(ValueError, match="ckpt_every"):
        api.check_ckpt(torch.zeros((0,) + tuple(u.shape), dtype=u.dtype), 10, 0, u)


def test_checkpoint_store_must_be_a_tensor():
    with pytest.raises(TypeError):
        api.check_ckpt([0.0] * 4, 10, 3, _state())


def test_fields_off_the_gpu_are_refused_before_the_library():
    # the first check of every entry point: a host tensor never reaches a
    # device pointer argument
    u = _state()
    with pytest.raises(ValueError, match="GPU"):
        api.run(u, u.clone(), dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1), 3, 0)
    with pytest.raises(ValueError, match="GPU"):
        api.adjoint_run(None, 1, u, u.clone(), dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1), 3, 0)
