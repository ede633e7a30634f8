"""GPU: gmt_nn_norm2_noalloc (partial sums in a fixed device array, no allocation)
against gmt_nn_norm2 through the C ABI: two calls in a row, the second with a
smaller input, and the size limit refused on the host side."""

import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2604_26518_amd import binding
    return binding


def _noalloc(x):
    B = _lib()
    out = ct.c_double()
    st = B.lib().gmt_nn_norm2_noalloc(ct.c_void_p(x.data_ptr()), ct.c_size_t(x.numel()), ct.byref(out),
                                      B._stream())
    return st, out.value


def test_noalloc_norm_matches_allocating_entry_point():
    B = _lib()
    fn = B.lib().gmt_nn_norm2_noalloc
    fn.argtypes = [ct.c_void_p, ct.c_size_t, ct.POINTER(ct.c_double), ct.c_void_p]
    fn.restype = ct.c_int
    rng = np.random.default_rng(7)
    # two calls in a row on the same device array, the second smaller: the first call's
    # partials beyond the second's grid must not leak into its sum
    for n in (5_000_003, 70_001, 1):
        x = torch.as_tensor(rng.standard_normal(n).astype(np.float32), device="cuda")
        st, got = _noalloc(x)
        assert st == 0, B.lib().gmt_last_error().decode()
        ref = B.norm2(x)
        exact = float((x.cpu().numpy().astype(np.float64) ** 2).sum())
        print(f"[noalloc] n={n}: {got!r} vs gmt_nn_norm2 {ref!r}", flush=True)
        assert abs(got - ref) <= 1e-13 * ref and abs(got - exact) <= 1e-12 * exact
    z = torch.zeros(4096, dtype=torch.float32, device="cuda")
    assert _noalloc(z) == (0, 0.0)


def test_noalloc_norm_rejects_oversize_input():
    B = _lib()
    fn = B.lib().gmt_nn_norm2_noalloc
    fn.argtypes = [ct.c_void_p, ct.c_size_t, ct.POINTER(ct.c_double), ct.c_void_p]
    fn.restype = ct.c_int
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = ct.c_double()
    # a size beyond the scratch limit is refused before any launch (the pointer is never read)
    st = fn(ct.c_void_p(x.data_ptr()), ct.c_size_t(8192 * 2048 + 1), ct.byref(out), B._stream())
    assert st == B.GMT_E_INVAL
    assert "exceeds" in B.lib().gmt_last_error().decode()
