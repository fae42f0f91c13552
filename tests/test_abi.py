"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, and validates parameters on the host without touching a GPU."""
import ctypes
import os
import re

import pytest

import scenarios

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_02107_amd", "libdnslab.so")


def header_symbols():
    text = open(os.path.join(ROOT, "include", "dnslab.h")).read()
    return sorted(set(re.findall(r"\b(dnslab_[a-z0-9_]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libdnslab.so not built")


@needs_lib
def test_every_header_symbol_is_exported():
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd._lib import EXPORTS
    lib = m.load()
    syms = header_symbols()
    assert syms == sorted(EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


@needs_lib
def test_workspace_bytes_and_validation():
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd._lib import DnslabError
    sc = scenarios.room(64, 32, 24, dx=0.05, n_boxes=1)
    b64 = m.workspace_bytes(sc, m.FP64)
    b32 = m.workspace_bytes(sc, m.FP32_REFINE)
    n = sc.ncells
    assert b64 > 13 * 8 * n and b32 > 13 * 4 * n and b32 < b64
    bad = sc.copy()
    bad.nx = 40          # 40 = 2^3 * 5 is not a supported FFT length
    with pytest.raises(DnslabError) as e:
        m.workspace_bytes(bad)
    assert e.value.code == -3
    bad = sc.copy()
    bad.tau_f = 0.0
    with pytest.raises(DnslabError) as e:
        m.workspace_bytes(bad)
    assert e.value.code == -1
    bad = sc.copy()
    bad.nx = 6
    bad.ny = 1
    bad.nz = 1
    assert m.workspace_bytes(bad) > 0


@needs_lib
def test_null_context_is_rejected_without_gpu():
    import paper_2204_02107_amd as m
    lib = m.load()
    assert lib.dnslab_step(None, 1, None) == -1
    assert lib.dnslab_poisson(None, None, None) == -1
    assert b"NULL" in lib.dnslab_last_error(None)
    lib.dnslab_destroy(None)


def test_header_documents_every_entry_point():
    text = open(os.path.join(ROOT, "include", "dnslab.h")).read()
    for s in header_symbols():
        m = re.search(r"\n(int|void|const char\*)\s+" + s + r"\(", text)
        assert m, s
        before = text[:m.start()].rstrip()
        # each declaration follows a comment, or shares one with the entry point above it
        assert before.endswith("*/") or before.endswith(");"), s


@needs_lib
def test_fft_length_limits():
    """Lines are staged whole in LDS: x up to 4096 (FP64) / 8192 (FP32), y and
    z up to 2048 / 4096; one step beyond is DNSLAB_EUNSUPPORTED."""
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd._lib import DnslabError
    base = scenarios.room(64, 32, 24, dx=0.05, n_boxes=1)

    def shaped(nx, ny, nz):
        c = base.copy()
        c.nx, c.ny, c.nz = nx, ny, nz
        return c
    ok = [((4096, 2, 2), m.FP64), ((8192, 2, 2), m.FP32_REFINE), ((4, 2048, 2), m.FP64),
          ((4, 2, 2048), m.FP64), ((4, 4096, 2), m.FP32_REFINE), ((4, 2, 4096), m.FP32_REFINE)]
    bad = [((4608, 2, 2), m.FP64), ((9216, 2, 2), m.FP32_REFINE), ((4, 2304, 2), m.FP64),
           ((4, 2, 4608), m.FP32_REFINE), ((2, 4, 4), m.FP64), ((4, 10, 4), m.FP64)]
    for shape, prec in ok:
        assert m.workspace_bytes(shaped(*shape), prec) > 0, shape
    for shape, prec in bad:
        with pytest.raises(DnslabError) as e:
            m.workspace_bytes(shaped(*shape), prec)
        assert e.value.code == -3, shape


@needs_lib
def test_allocator_pair_must_be_complete():
    """alloc and free_ are both set or both NULL (host-side validation)."""
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd import _lib
    sc = scenarios.room(64, 32, 24, dx=0.05, n_boxes=1)
    lib = m.load()
    P = m.make_params(sc)
    out = ctypes.c_size_t()
    assert lib.dnslab_workspace_bytes(ctypes.byref(P), ctypes.byref(out)) == 0
    P.alloc = _lib.TORCH_ALLOC
    assert lib.dnslab_workspace_bytes(ctypes.byref(P), ctypes.byref(out)) == -1
    assert b"alloc" in lib.dnslab_last_error(None)
    P.free_ = _lib.TORCH_FREE
    assert lib.dnslab_workspace_bytes(ctypes.byref(P), ctypes.byref(out)) == 0
    h = ctypes.c_void_p()
    assert lib.dnslab_pool_create(1 << 20, 0, None, _lib.TORCH_ALLOC, _lib.FREE_FN(), None, ctypes.byref(h)) == -1
    assert not h.value


def test_params_struct_matches_header_field_order():
    """The ctypes mirror of dnslab_params lists the header's fields in order."""
    from paper_2204_02107_amd._lib import Params
    text = open(os.path.join(ROOT, "include", "dnslab.h")).read()
    body = text[text.index("typedef struct {\n    int32_t nx, ny, nz;"):text.index("} dnslab_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.split("{", 1)[-1].strip()
        if not decl:
            continue
        fn = re.match(r".*\(\s*\*\s*(\w+)\s*\)", decl, flags=re.S)
        if fn:
            names.append(fn.group(1))
            continue
        for part in decl.split(","):
            nm = re.findall(r"(\w+)\s*(\[\d+\])?\s*$", part.strip())
            if nm:
                names.append(nm[0][0])
    assert names == [f[0] for f in Params._fields_]
