"""Host-side checks of the C ABI (no GPU needed): symbols, size queries, argument errors."""
import ctypes as C
import os
import re

import pytest

from paper_2508_07193_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "flashmp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)       # declarations only, not comments
    return sorted(set(re.findall(r"\b(fmp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib.load()


def test_exports_every_declared_symbol(L):
    declared = _header_symbols()
    assert set(declared) == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def _desc(n=64, sub=32, c=2.0):
    d = _lib.DomainDesc()
    d.nx = d.ny = d.nz = n
    d.c = c
    d.eps_block = None
    d.eps_block_size = 0
    d.sub_x = d.sub_y = d.sub_z = sub
    return d


def _size(L, descs, overlap=1, prec=0):
    arr = (_lib.DomainDesc * len(descs))(*descs)
    pd = _lib.PrecondDesc(overlap, prec, 0, 0)
    nb = C.c_size_t(0)
    h = C.c_void_p()
    st = L.fmp_setup_subdomains(arr, len(descs), C.byref(pd), None, C.byref(nb), None, C.byref(h))
    return st, nb.value


def test_workspace_query_runs_on_host(L):
    st, nb = _size(L, [_desc()])
    assert st == 0
    # staging for 8 boxes of side 33 (each touches three walls) in FP64 plus tables
    assert nb >= 3 * 8 * 33**3 * 8
    st32, nb32 = _size(L, [_desc()], prec=1)
    assert st32 == 0 and nb32 < nb


@pytest.mark.parametrize("kw,want", [
    (dict(overlap=0), -1),            # overlap must be >= 1
    (dict(n=30, sub=32), -1),         # sub must divide the side
    (dict(n=1, sub=0), -1),           # side < 2
])
def test_invalid_descriptors(L, kw, want):
    overlap = kw.pop("overlap", 1)
    st, _ = _size(L, [_desc(**kw)], overlap=overlap)
    assert st == want


def test_oversized_boxes_still_get_a_workspace_size(L):
    # box side 128 exceeds the largest transform class: setup sizes the stencil-only handle
    st, nb = _size(L, [_desc(n=128, sub=128)])
    assert st == 0 and 0 < nb < 3 * 128**3 * 8
    # boxes of 65 cells run the large-box path, whose FP64 staging holds two copies
    st, nb = _size(L, [_desc(n=128, sub=64)])
    assert st == 0 and nb >= 2 * 3 * 8 * 65**3 * 8


def test_status_strings(L):
    assert L.fmp_status_string(0) == b"ok"
    assert L.fmp_status_string(-2) == b"input and output overlap"


def _size_pd(L, descs, pd):
    arr = (_lib.DomainDesc * len(descs))(*descs)
    nb = C.c_size_t(0)
    h = C.c_void_p()
    st = L.fmp_setup_subdomains(arr, len(descs), C.byref(pd), None, C.byref(nb), None, C.byref(h))
    return st, nb.value


def test_index_block_workspace_query(L):
    # 64^3 in 32^3 index blocks, overlap 0: eight wall patterns, eight C^{-1}
    # of order 6n^2 - 3n = 6048 (padded to 6080), Table II's dense matrix each
    st, nb = _size_pd(L, [_desc(64, 32)], _lib.PrecondDesc(0, 0, 0, 0, 0, 1))
    assert st == 0
    assert nb >= 8 * 6080 * 6080 * 8
    # overlap 0 is admissible for index blocks only
    st, _ = _size_pd(L, [_desc(64, 32)], _lib.PrecondDesc(0, 0, 0, 0, 0, 0))
    assert st == -1
    # FP32 transforms, the learned part and the autotuner are PEC-box features
    for pd in (_lib.PrecondDesc(0, 1, 0, 0, 0, 1), _lib.PrecondDesc(0, 0, 1, 0, 0, 1),
               _lib.PrecondDesc(0, 0, 0, -1, 0, 1)):
        st, _ = _size_pd(L, [_desc(64, 32)], pd)
        assert st == -6
    st, _ = _size_pd(L, [_desc(64, 32)], _lib.PrecondDesc(0, 0, 0, 0, 0, 2))
    assert st == -1


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Every struct the binding passes across the ABI has the size and field
    offsets the C compiler gives it (a mismatch would make the library read
    or write past the caller's host memory)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fmp_domain_desc": _lib.DomainDesc, "fmp_precond_desc": _lib.PrecondDesc,
               "fmp_tune_entry": _lib.TuneEntry, "fmp_solve_opts": _lib.SolveOpts,
               "fmp_solve_info": _lib.SolveInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "flashmp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_bf16_refuses_planes_beyond_its_32bit_slab_offsets(L):
    # the bf16 gather addresses a 4-plane slab by 32-bit byte offsets:
    # planes of 2^27 cells or more are refused at setup, in bf16 only
    def flat(nx, ny):
        d = _desc(n=2, sub=0)
        d.nx, d.ny = nx, ny
        return d
    st, _ = _size(L, [flat(16384, 8192)], prec=2)        # 2^27 cells per plane
    assert st == -6
    st, _ = _size(L, [flat(16384, 8192)], prec=0)
    assert st == 0
    st, _ = _size(L, [flat(8192, 8192)], prec=2)         # 2^26: within range
    assert st == 0


def test_eps_table_shape_is_checked_before_the_library_reads_it():
    # the library reads ceil(n / b) cubes per axis from the host table: the
    # binding refuses any other shape instead of letting it read past the array
    import numpy as np
    from paper_2508_07193_amd import api, inputs
    rng = np.random.default_rng(0)
    eps = inputs.eps_table(rng, 70, 37, 21, 4)
    assert eps.shape == (6, 10, 18)
    d, keep = api.domain_desc(70, 37, 21, 2.0, eps=eps, eps_block=4)
    assert d.eps_block_size == 4 and keep.shape == (6, 10, 18)
    with pytest.raises(ValueError, match="expected"):
        api.domain_desc(70, 37, 21, 2.0, eps=eps[:5, :9, :17], eps_block=4)
    with pytest.raises(ValueError, match="expected"):
        api.domain_desc(70, 37, 21, 2.0, eps=eps, eps_block=0)
