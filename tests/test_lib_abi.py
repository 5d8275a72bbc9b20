"""The C-ABI library loads and exports every symbol include/nematic_sph.h
declares; host-only entry points work without a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "nematic_sph.h")).read()
    names = set(re.findall(r"\b(nem_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_header_matches_binding():
    import paper_2108_08919_amd as P
    assert set(header_symbols()) == set(P.EXPORTED)


def test_library_exports_every_symbol():
    import ctypes
    import paper_2108_08919_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(P.LIB_PATH)
    for name in header_symbols():
        assert hasattr(L, name), name


def test_host_only_calls():
    import paper_2108_08919_amd as P
    import workloads as wl
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    assert P.nem_version() >= 100
    assert "invalid" in P.strerror(P.NEM_E_INVAL)
    p = wl.config("C1")["params"]
    b = P.nem_arena_bytes([p], [4096])
    assert b > 4096 * 100
    b2 = P.nem_arena_bytes([p, p.replace(L=128.0)], [4096, 128 * 128])
    assert b2 > b
    with pytest.raises(P.NemError) as e:
        P.nem_arena_bytes([p.replace(L=8.0)], [64])          # fewer than three cells per side
    assert e.value.code == P.NEM_E_INVAL
    with pytest.raises(P.NemError):
        P.nem_arena_bytes([p.replace(form=1, elastic=1)], [4096])
    with pytest.raises(P.NemError):
        P.nem_arena_bytes([p], [0])


def test_replicas_must_share_the_compiled_variant():
    """One launch per pass serves every replica: form, elastic and kernel must
    agree across replicas, and the kernel must be 0 or 1 (host-side check)."""
    import paper_2108_08919_amd as P
    import workloads as wl
    p0 = wl.Params(L=32.0)
    for ps in ([p0, p0.replace(kernel=1)], [p0, p0.replace(form=1)], [p0, p0.replace(elastic=1)],
               [p0.replace(kernel=2)]):
        with pytest.raises(P.NemError):
            P.nem_arena_bytes(ps, [1024] * len(ps))
    assert P.nem_arena_bytes([p0.replace(kernel=1)] * 2, [1024, 2048]) > 0
