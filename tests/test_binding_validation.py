"""The Python binding rejects tensors that cannot be handed to the C ABI (host memory,
wrong dtype, strided views, another device) before any pointer reaches the library.
Host-only: the context object is built without a device."""
import pytest
import torch

from paper_2009_04755_amd import Clouds, Context, SparseSet, _lib


@pytest.fixture
def ctx():
    c = object.__new__(Context)  # no rocket_create: these checks never reach the library
    c.device = 0
    c.handle = None
    return c


def test_sparse_set_on_host_rejected(ctx):
    S = SparseSet(torch.tensor([0, 2, 3]), torch.tensor([1, 5, 7]), torch.ones(3))
    with pytest.raises(ValueError, match="device tensor"):
        ctx._items(S, _lib.SPARSE_COSINE)


def test_wrong_dtype_rejected(ctx):
    with pytest.raises(TypeError, match="keys"):
        ctx._dev(torch.tensor([1, 5, 7], dtype=torch.int32), "keys", torch.int64)


def test_clouds_offsets_on_host_rejected(ctx):
    cl = Clouds(torch.tensor([0, 1, 2]), torch.zeros(4), 0.02)
    with pytest.raises(ValueError, match="offsets"):
        ctx._items(cl, _lib.GAUSS_OVERLAP)


def test_dense_on_host_rejected(ctx):
    with pytest.raises(ValueError, match="device tensor"):
        ctx._items(torch.zeros(4, 8), _lib.NCC_BF16X6)


def test_not_a_tensor_rejected(ctx):
    with pytest.raises(TypeError):
        ctx._items([[0.0] * 8] * 4, _lib.NCC_FP32)
    with pytest.raises(TypeError):
        ctx._items(torch.zeros(4, 8), _lib.SPARSE_COSINE)


def test_strided_view_rejected_by_contiguity_check(ctx):
    # the contiguity check runs after the device check; exercise it on a meta-device stand-in
    t = torch.empty(10, dtype=torch.int64, device="meta")[::2]
    with pytest.raises(ValueError):
        ctx._dev(t, "keys", torch.int64)


def test_host_items_must_be_cpu_float32(ctx):
    with pytest.raises(ValueError):
        ctx.allpairs_host(torch.zeros(4, 8, dtype=torch.float64))
