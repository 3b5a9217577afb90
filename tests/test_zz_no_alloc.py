"""The no-allocation sort entry point (vrs_sort_pairs_noalloc, workspace in a
fixed device array of the library) against the workspace sort it shares its
kernels with (vrs_sort_pairs), called through the C ABI: two calls in a row,
the second smaller, bit-identical results, both equal to NumPy's stable
sort."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pairs(rng, n, bits, dups):
    hi = (1 << bits) - 1 if bits < 64 else (1 << 64) - 1
    base = rng.integers(0, hi, size=max(n // dups, 1), dtype=np.uint64, endpoint=True)
    keys = base[rng.integers(0, len(base), size=n)]
    vals = rng.permutation(n).astype(np.uint32)
    return keys, vals


def _to_gpu(keys, vals, cap):
    kt = torch.zeros(cap, dtype=torch.int64, device="cuda")
    vt = torch.zeros(cap, dtype=torch.int32, device="cuda")
    kt[:len(keys)] = torch.from_numpy(keys.view(np.int64)).cuda()
    vt[:len(vals)] = torch.from_numpy(vals.view(np.int32)).cuda()
    return kt, vt


def test_noalloc_sort_equals_workspace_sort_twice():
    from paper_2505_10144_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(77)
    cases = [(L.VRS_SORT_NOALLOC_MAX_PAIRS - 5, L.VRS_SORT_NOALLOC_MAX_PAIRS, 46, 3),
             (100_003, 150_000, 40, 50)]
    for n, cap, bits, dups in cases:
        print(f"[noalloc] n={n} capacity={cap} bits={bits}", flush=True)
        keys, vals = _pairs(rng, n, bits, dups)
        nt = torch.tensor([n], dtype=torch.int32, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        # Reference: the workspace entry point.
        k1, v1 = _to_gpu(keys, vals, cap)
        ws = torch.empty(int(lib.vrs_sort_pairs_workspace_size(cap)), dtype=torch.uint8, device="cuda")
        rc = lib.vrs_sort_pairs(ctypes.c_void_p(k1.data_ptr()), ctypes.c_void_p(v1.data_ptr()),
                                ctypes.c_void_p(nt.data_ptr()), cap, bits, ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), ctypes.c_void_p(st.data_ptr()), _stream())
        assert rc == 0
        # The no-allocation entry point.
        k2, v2 = _to_gpu(keys, vals, cap)
        rc = lib.vrs_sort_pairs_noalloc(ctypes.c_void_p(k2.data_ptr()), ctypes.c_void_p(v2.data_ptr()),
                                        ctypes.c_void_p(nt.data_ptr()), cap, bits,
                                        ctypes.c_void_p(st.data_ptr()), _stream())
        assert rc == 0
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert torch.equal(k1, k2) and torch.equal(v1, v2)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(k2[:n].cpu().numpy().view(np.uint64), keys[order])
        assert np.array_equal(v2[:n].cpu().numpy().view(np.uint32), vals[order])
        assert bool((k2[n:] == 0).all()) and bool((v2[n:] == 0).all())
