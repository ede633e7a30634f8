"""GPU: gmt_nn_norm2_noalloc (partial sums in the library's fixed device array, no
allocation) against gmt_nn_norm2 through the C ABI: calls in a row on one device, each
smaller than the one before, and the size limit refused on the host side."""

import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2604_26518_amd import binding
    return binding


def _noalloc(x, n=None):
    B = _lib()
    out = ct.c_double()
    st = B.lib().gmt_nn_norm2_noalloc(ct.c_void_p(x.data_ptr()), ct.c_size_t(x.numel() if n is None else n),
                                      ct.byref(out), B._stream())
    return st, out.value


def test_noalloc_norm_matches_allocating_entry_point():
    B = _lib()
    rng = np.random.default_rng(7)
    # calls in a row on the same device array, each smaller than the last: the earlier
    # call's partials beyond the later one's grid must not leak into its sum
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
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    # a size beyond the fixed array's limit is refused before any launch (the pointer is never read)
    st, _ = _noalloc(x, 8192 * 2048 + 1)
    assert st == B.GMT_E_INVAL
    assert "exceeds" in B.lib().gmt_last_error().decode()
