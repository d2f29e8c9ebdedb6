"""The allocation-free relative L2 (pf_rel_l2_noalloc) against pf_rel_l2,
called through the C ABI: two calls in a row, the second on a smaller
input, both bit-identical to the allocating entry point and within 1e-14 of
the definition; argument errors."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_rel_l2_matches_the_allocating_entry_point():
    import torch
    from paper_2609_36100_amd import _lib
    _say("pf_rel_l2_noalloc")
    L = _lib.lib()
    rng = np.random.default_rng(31)
    for n in (3_000_001, 4097):            # a large call, then a smaller one
        a_h = rng.standard_normal(n)
        b_h = a_h + 1e-3 * rng.standard_normal(n)
        a = torch.from_numpy(a_h).cuda()
        b = torch.from_numpy(b_h).cuda()
        torch.cuda.synchronize()
        got, ref = ctypes.c_double(), ctypes.c_double()
        assert L.pf_rel_l2_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, None,
                                   ctypes.byref(got)) == 0
        assert L.pf_rel_l2(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, None,
                           ctypes.byref(ref)) == 0
        assert got.value == ref.value, (n, got.value, ref.value)
        defn = np.linalg.norm(a_h - b_h) / np.linalg.norm(b_h)
        assert abs(got.value - defn) <= 1e-14 * defn
    z = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert L.pf_rel_l2_noalloc(ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()), 0, None,
                               ctypes.byref(got)) == -1
    assert L.pf_rel_l2_noalloc(None, ctypes.c_void_p(z.data_ptr()), 16, None, ctypes.byref(got)) == -1
    assert L.pf_rel_l2_noalloc(ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()), (1 << 41) + 1, None,
                               ctypes.byref(got)) == -1
