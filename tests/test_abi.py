"""CPU-side checks of the C ABI: the library loads, exports every declared entry point, and rejects
invalid arguments before touching the device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            if not m.group(0).lstrip().startswith(("typedef", "#", "enum", "struct")):
                names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_2010_10638_amd as tk
    return tk.load_library()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("tucker_init", "ttmc_mode", "qrp_update", "hooi_sweep", "reconstruct", "tucker_free"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def _init(lib, order=3, dims=(5, 6, 7), ranks=(2, 2, 2), nnz=0, dtype=1, flags=0, out=True):
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * max(order, 1))(*[int(x) for x in dims][:max(order, 1)]) if dims is not None else None
    r = (ctypes.c_int32 * max(order, 1))(*[int(x) for x in ranks][:max(order, 1)]) if ranks is not None else None
    return lib.tucker_init(ctypes.byref(h) if out else None, order, d, r, nnz, None, None, dtype, flags, None)


@pytest.mark.parametrize("kw,code", [
    (dict(out=False), 1),
    (dict(order=1, dims=(5,), ranks=(2,)), 1),
    (dict(order=9, dims=(2,) * 9, ranks=(1,) * 9), 1),
    (dict(dims=None), 1),
    (dict(dtype=7), 1),
    (dict(nnz=-1), 1),
    (dict(nnz=1 << 31), 5),
    (dict(nnz=10), 1),                                   # coords/vals null
    (dict(flags=0x80), 1),
    (dict(flags=0x10), 1),                               # the first bit past TK_FLAG_NO_MEMO
    (dict(ranks=(6, 2, 2)), 1),                          # R_1 > I_1
    (dict(dims=(5, 0, 7)), 1),
    (dict(dims=(2000,) * 3, ranks=(65, 65, 65)), 5),     # K_n = 4225 > 4096
    (dict(dims=(50, 50, 50), ranks=(10, 2, 3)), 1),      # R_1 = 10 > K_1 = 6
    (dict(dims=(1 << 30, 1 << 30, 1 << 4), ranks=(1, 1, 1)), 5),  # prod dims >= 2^63
])
def test_init_rejects_invalid_arguments(lib, kw, code):
    assert _init(lib, **kw) == code
    assert len(lib.tucker_last_error()) > 0


def test_null_context_is_rejected(lib):
    assert lib.ttmc_mode(None, 0, None, None, None) == 1
    assert lib.qrp_update(None, 0, None, None, None, None) == 1
    assert lib.hooi_sweep(None, None, None, None, None, None) == 1
    assert lib.reconstruct(None, None, None, 0, None, None, None) == 1
    assert lib.svd_update(None, 0, None, None, None) == 1
    assert lib.tucker_svd_info(None, None) == 1
    assert lib.hooi_run(None, None, None, 1, ctypes.c_double(0.0), None, None, None) == 1
    lib.tucker_free(None)


def test_product_and_oracle_are_independent():
    """The GPU package never names the oracle, and the oracle never names the GPU package."""
    for d, other in (("paper_2010_10638_amd", "oracle"), ("oracle", "paper_2010_10638_amd")):
        for base, _, files in os.walk(os.path.join(ROOT, d)):
            for f in files:
                if f.endswith((".py", ".c", ".h", ".hip", ".cpp")):
                    text = open(os.path.join(base, f)).read()
                    assert not re.search(rf"\b(import|from)\s+{other}\b", text), (f, other)
                    if d == "paper_2010_10638_amd":
                        assert "oracle" not in text.lower(), f


def _kernel(lib, dims, ranks, dtype, mode):
    N = len(dims)
    d = (ctypes.c_int64 * N)(*dims)
    r = (ctypes.c_int32 * N)(*ranks)
    k = ctypes.c_int(-1)
    assert lib.tucker_ttmc_kernel(N, d, r, dtype, mode, ctypes.byref(k)) == 0
    return k.value


@pytest.mark.parametrize("dtype,limit", [(1, 1 << 25), (2, 1 << 26), (0, 1 << 24)])
def test_order3_kernel_only_below_32bit_offsets(lib, dtype, limit):
    """The order-3 matrix-core kernel forms gather offsets in 32 bits: a mode takes it only while
    every other factor copy (I_t x 16 columns) stays below 2^31 bytes; at the limit the generic
    kernel (64-bit offsets) runs instead.  Host-only query, no device needed."""
    GENERIC, ORDER3 = 0, 1
    assert _kernel(lib, [1000, limit - 1, 500], [8, 8, 8], dtype, 0) == ORDER3
    assert _kernel(lib, [1000, limit, 500], [8, 8, 8], dtype, 0) == GENERIC
    assert _kernel(lib, [1000, limit, 500], [8, 8, 8], dtype, 1) == ORDER3    # mode 1 does not gather U_1
    assert _kernel(lib, [1000, 900, 500], [17, 8, 8], dtype, 1) == GENERIC   # R above 16


def test_kernel_choice_by_order(lib):
    GENERIC, FIBER = 0, 2
    assert _kernel(lib, [50, 50, 50, 50], [8, 8, 8, 8], 1, 0) == FIBER
    assert _kernel(lib, [50, 50, 50, 50], [4, 12, 12, 16], 1, 3) == FIBER
    assert _kernel(lib, [30, 30, 30, 30], [20, 3, 4, 5], 1, 1) == GENERIC     # inner rank above 16
    assert _kernel(lib, [9] * 6, [2] * 6, 1, 0) == GENERIC
    assert _kernel(lib, [300, 250], [6, 6], 1, 0) == GENERIC
    k = ctypes.c_int()
    d = (ctypes.c_int64 * 3)(5, 5, 5)
    r = (ctypes.c_int32 * 3)(2, 2, 2)
    assert lib.tucker_ttmc_kernel(3, d, r, 1, 3, ctypes.byref(k)) == 1        # mode out of range
    assert lib.tucker_ttmc_kernel(3, d, r, 9, 0, ctypes.byref(k)) == 1        # unknown dtype
