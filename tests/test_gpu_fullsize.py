"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (the library's persistent default grid).

* n = 2^28 binary64, cancelling pairs + 1% perturbations: the GPU result
  equals the oracle's, and the oracle's exact total equals the closed form
  (the sum of the replaced pairs only).
* n = 2^31 binary64 (16 GiB), N(0,1) * 2^k with subnormals and balanced
  +-DBL_MAX: exact result; with unbalanced +-DBL_MAX the sum overflows, and
  the exported exact state still equals the oracle's integer.
"""

import gc

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import gpu_sum_async

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)


def _device(bits):
    import torch
    return torch.from_numpy(bits.view(np.int64)).to("cuda")


def _release():
    import torch
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", ["a", "b"])
def test_config2_full_size(variant):
    print("config2 variant", variant, "n=2^28", flush=True)
    bits, terms = workloads.config2(log2n=28, seed=0, variant=variant)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    assert acc.total == oracle.exact_sum_binned(terms, "f64")[0].total
    x = _device(bits)
    got = gpu_sum_async(x, len(bits), "f64")
    assert got[:2] == tuple(oracle.finish(acc, "f64"))
    assert got[2] == bytes(576)
    del x
    _release()


def test_config3_full_size_balanced():
    n = 1 << 31
    print("config3 balanced n=2^31", flush=True)
    bits = workloads.config3(n=n, seed=0)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    x = _device(bits)
    del bits
    got = gpu_sum_async(x, n, "f64")
    assert got[:2] == tuple(oracle.finish(acc, "f64"))
    del x
    _release()


def test_config3_full_size_overflow_state():
    import torch
    import paper_1605_05436_amd as xs
    n = 1 << 31
    print("config3 unbalanced n=2^31", flush=True)
    bits = workloads.config3(n=n, seed=0, balanced=False)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    x = _device(bits)
    del bits
    got = gpu_sum_async(x, n, "f64")
    want = tuple(oracle.finish(acc, "f64"))
    assert got[:2] == want
    assert want[1] & oracle.FLAG_OVERFLOW
    st = xs.new_states(1)
    xs.xsum_acc_add(st.data_ptr(), x.data_ptr(), n, xs.F64, xs.stream_handle())
    torch.cuda.synchronize()
    raw = st.cpu().numpy().reshape(-1)
    digits = raw[:68 * 8].view(np.int64).tolist()
    assert sum(d << (32 * j) for j, d in enumerate(digits)) == acc.total
    del x
    _release()
