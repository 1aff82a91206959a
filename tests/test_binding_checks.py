"""The Python binding refuses bad arguments before any call into the library (CPU only).

A stand-in object with the attributes of a device tensor exercises the checks on
x and y, since no device tensors exist without a GPU.
"""
import numpy as np
import pytest
import torch

import paper_2302_05662_amd as S
from paper_2302_05662_amd import spmv as B


class FakeDeviceTensor:
    """Just the metadata the binding inspects on a device tensor."""

    is_cuda = True

    def __init__(self, n, dtype=torch.float32, contiguous=True, device=0):
        self._n, self.dtype, self._contig = n, dtype, contiguous
        self.device = torch.device("cuda", device)

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        return 0x1000


def _handle(n_rows=100, n_cols=80, dtype_code=S.SPMV_F32):
    # ptr None: no library handle behind it, so nothing is ever freed or run
    return B.Handle(None, n_rows, n_cols, 500, dtype_code, device=0)


@pytest.mark.parametrize("bad,msg", [
    (dict(x=FakeDeviceTensor(79)), "elements"),                       # x shorter than n_cols
    (dict(y=FakeDeviceTensor(99)), "elements"),                       # y shorter than n_rows
    (dict(x=FakeDeviceTensor(80, torch.float64)), "dtype"),           # FP64 x on an FP32 matrix
    (dict(y=FakeDeviceTensor(100, torch.float16)), "dtype"),
    (dict(x=FakeDeviceTensor(80, contiguous=False)), "contiguous"),
    (dict(y=FakeDeviceTensor(100, device=1)), "device"),              # another GPU
    (dict(x=torch.zeros(80)), "device tensor"),                       # host tensor
    (dict(y=np.zeros(100, np.float32)), "device tensor"),
])
def test_run_time_tune_refuse_bad_vectors(bad, msg):
    h = _handle()
    args = dict(x=FakeDeviceTensor(80), y=FakeDeviceTensor(100))
    args.update(bad)
    for call in (lambda: S.spmv_run(h, S.SPMV_FMT_CSR, 1.0, args["x"], 0.0, args["y"]),
                 lambda: S.spmv_time(h, S.SPMV_FMT_CSR, args["x"], args["y"]),
                 lambda: S.spmv_tune(h, S.SPMV_FMT_CSR, args["x"], args["y"])):
        with pytest.raises(ValueError, match=msg):
            call()


def test_fp64_handle_wants_fp64_vectors():
    h = _handle(dtype_code=S.SPMV_F64)
    with pytest.raises(ValueError, match="dtype"):
        S.spmv_run(h, S.SPMV_FMT_CSR, 1.0, FakeDeviceTensor(80, torch.float32), 0.0,
                   FakeDeviceTensor(100, torch.float64))


def test_create_refuses_bad_index_arrays():
    v = np.ones(3, np.float32)
    with pytest.raises(ValueError, match="int32"):  # int64 tensors are not reinterpreted
        S.spmv_create(4, 4, torch.arange(3), torch.arange(3, dtype=torch.int32), torch.ones(3))
    with pytest.raises(ValueError, match="range"):  # would wrap to a valid index
        S.spmv_create(4, 4, np.array([0, 1, 2**32 + 2]), np.arange(3), v)
    with pytest.raises(ValueError, match="integer"):
        S.spmv_create(4, 4, np.array([0.0, 1.0, 2.0]), np.arange(3), v)
    with pytest.raises(ValueError, match="same length"):
        S.spmv_create(4, 4, np.arange(3), np.arange(2), v)
    with pytest.raises(ValueError, match="unsupported"):
        S.spmv_create(4, 4, np.arange(3), np.arange(3), np.ones(3, np.float16))


def test_batch_wrappers_check_each_vector():
    hs = [_handle(10, 8), _handle(20, 16)]
    good_x = [FakeDeviceTensor(8), FakeDeviceTensor(16)]
    good_y = [FakeDeviceTensor(10), FakeDeviceTensor(20)]
    with pytest.raises(ValueError, match=r"xs\[1\].*elements"):
        S.spmv_batch_create(hs, [good_x[0], FakeDeviceTensor(15)], good_y)
    with pytest.raises(ValueError, match=r"ys\[0\].*dtype"):
        S.spmv_batch_create(hs, good_x, [FakeDeviceTensor(10, torch.float64), good_y[1]])
    with pytest.raises(ValueError, match="entries"):
        S.spmv_batch_create(hs, good_x[:1], good_y)
    with pytest.raises(ValueError, match="alphas"):
        S.spmv_batch_create(hs, good_x, good_y, alphas=[1.0])
    b = B.Batch(None, hs, good_x, good_y)  # no library batch behind it
    with pytest.raises(ValueError, match=r"ys\[1\].*elements"):
        S.spmv_batch_run(b, ys=[good_y[0], FakeDeviceTensor(19)])
    with pytest.raises(ValueError, match=r"xs\[0\].*device tensor"):
        S.spmv_batch_update(b, xs=[torch.zeros(8), good_x[1]])
    with pytest.raises(ValueError, match="betas"):
        S.spmv_batch_run(b, betas=[0.0, 0.0, 0.0])
