"""The allocation-free marking entry (dpg_dorfler_mark_noalloc) through the
C ABI against dpg_dorfler_mark: bit-exact flags on two calls in a row, the
second with a smaller input (the static scratch keeps the first call's
contents), and the size limit rejected on the host."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2609_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _values(n, seed):
    rng = np.random.default_rng(W.SEED_BASE + seed)
    v = np.exp(rng.standard_normal(n) * 2.0)
    v[rng.choice(n, n // 50, replace=False)] = 0.0            # zeros tie
    v[: n // 100] = v[n // 100: 2 * (n // 100)]                 # repeated values
    return v


def test_noalloc_marking_matches_allocating_entry():
    torch = _torch()
    from paper_2609_03155_amd import dpg
    L = dpg.lib()
    stream = torch.cuda.current_stream()
    for n, seed, fr, fc in ((1 << 20, 91, 0.30, 0.05), (100003, 92, 0.5, 0.1)):
        print(f"case: dorfler_mark_noalloc n={n} seed={seed}", flush=True)
        sys.stdout.flush()
        v = torch.from_numpy(_values(n, seed)).cuda()
        ref = torch.full((n,), 9, dtype=torch.int8, device="cuda")
        got = torch.full((n,), 9, dtype=torch.int8, device="cuda")
        assert L.dpg_dorfler_mark(n, v.data_ptr(), fr, fc, ref.data_ptr(), None, 0, stream.cuda_stream) == dpg.DPG_OK
        rc = L.dpg_dorfler_mark_noalloc(n, v.data_ptr(), fr, fc, got.data_ptr(), stream.cuda_stream)
        assert rc == dpg.DPG_OK, L.dpg_last_error()
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(r, g)
        assert (r == 1).any() and (r == -1).any() and (r == 0).any()


def test_noalloc_marking_rejects_sizes_beyond_its_scratch():
    _torch()
    from paper_2609_03155_amd import dpg
    L = dpg.lib()
    # rejected on the host before any device access (the pointers are never read)
    assert L.dpg_dorfler_mark_noalloc((1 << 20) + 1, C.c_void_p(8), 0.3, 0.05, C.c_void_p(8), None) == \
        dpg.DPG_ERR_UNSUPPORTED
    assert L.dpg_dorfler_mark_noalloc(0, None, 0.3, 0.05, None, None) == dpg.DPG_OK
    assert L.dpg_dorfler_mark_noalloc(5, None, 0.3, 0.05, None, None) == dpg.DPG_ERR_ARG
