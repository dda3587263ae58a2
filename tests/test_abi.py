"""The C-ABI library loads and exports every function include/md.h declares; host-side
argument checks and layout queries (no GPU needed for these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1507_07068_amd import build as B
from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if B.is_stale():
        B.build_library()
    return md.load_library()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "md.h")).read()
    return re.findall(r"MD_API\s+[\w\s\*]+?\b(md_\w+)\s*\(", txt)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("md_build_neighbors", "md_eam_forces", "md_morse_forces", "md_verlet_step",
                     "md_energy"):
        assert required in names
    assert sorted(names) == sorted(md.API)


def test_library_exports_every_declared_symbol(lib):
    raw = C.CDLL(md.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_struct_sizes_match_header(lib):
    assert C.sizeof(md.Params) == 6 * 8 + 4 * 8 + 4 * 8 + 4 * 4 + 2 * 4 + 14 * 8 + 2 * 4
    assert C.sizeof(md.ReplicaDesc) == 6 * 8 + 6 * 4
    assert C.sizeof(md.Atoms) == 6 * 8
    assert C.sizeof(md.Lists) == 6 * 8
    assert C.sizeof(md.Status) == 8 * 4


def test_binding_constants_match_header():
    """Every integer #define of include/md.h that the binding also names has the same value."""
    txt = open(os.path.join(ROOT, "include", "md.h")).read()
    seen = 0
    for name, val in re.findall(r"#define\s+(MD_\w+)\s+(\(?[0-9x<\s]+\)?)\s", txt):
        if hasattr(md, name):
            assert getattr(md, name) == eval(val, {}), name
            seen += 1
    assert seen >= 20
    for name in ("MD_E_EMBED", "MD_F_IND_X", "MD_IND_Z", "MD_NBUILDS", "MD_TRACE_EVENTS", "MD_SCRATCH_BYTES"):
        assert hasattr(md, name), name


STRUCTS = {"md_params": md.Params, "md_replica_desc": md.ReplicaDesc, "md_atoms": md.Atoms,
           "md_lists": md.Lists, "md_status": md.Status, "md_trace": md.Trace,
           "md_eam_params": md.EamParams, "md_morse_params": md.MorseParams,
           "md_eam_paper_params": md.PaperParams}


def test_binding_layout_matches_header(tmp_path):
    """Every field offset and struct size of the Python binding equals what a C compiler makes
    of include/md.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "md.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} . %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            cname, fname, v = ln.split()
            got[(cname, fname)] = int(v)
    for cname, cls in STRUCTS.items():
        assert got[(cname, ".")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def _create(lib, systems, cap=64, xcap=64):
    descs = (md.ReplicaDesc * len(systems))(*[md.make_replica_desc(s) for s in systems])
    p = md.make_params(systems[0], cap, xcap)
    h = C.c_void_p()
    rc = lib.md_system_create(C.cast(descs, C.c_void_p), len(systems), C.byref(p), C.byref(h))
    return rc, h


def test_create_layout_and_padding(lib):
    reps = [I.replica(r) for r in range(3)]
    rc, h = _create(lib, reps)
    assert rc == md.MD_OK and h.value
    offs = [lib.md_replica_offset(h, r) for r in range(3)]
    assert offs[0] == 0
    for r in range(2):
        assert offs[r + 1] - offs[r] >= reps[r].n
        assert (offs[r + 1] - offs[r]) % md.MD_TILE == 0
    assert lib.md_system_atoms(h) >= sum(s.n for s in reps)
    assert lib.md_system_carbons(h) == sum(s.n_c for s in reps)
    assert lib.md_workspace_bytes(h) > 0
    assert lib.md_replica_offset(h, 3) == -1
    lib.md_system_destroy(h)


def test_create_rejects_bad_arguments(lib):
    s = I.bulk(4)
    assert _create(lib, [s], cap=0)[0] == md.MD_ERR_ARG
    small = I.bulk(2)    # 5.77 A periodic box: shorter than twice the list radius
    assert _create(lib, [small])[0] == md.MD_ERR_ARG
    bad = s.copy()
    bad.box_len = np.array([10.0, -1.0, 10.0])
    assert _create(lib, [bad])[0] == md.MD_ERR_ARG
    h = C.c_void_p()
    assert lib.md_system_create(None, 1, None, C.byref(h)) == md.MD_ERR_ARG


def test_calls_without_workspace_are_refused(lib):
    s = I.bulk(4)
    rc, h = _create(lib, [s])
    assert rc == md.MD_OK
    a, l = md.Atoms(1, 1, 1, 1, 1, 1), md.Lists(1, 1, 1, 1)
    assert lib.md_build_neighbors(h, C.byref(a), C.byref(l), 0, None) == md.MD_ERR_STATE
    assert lib.md_eam_forces(h, C.byref(a), C.byref(l), md.MD_F_FORCE, None, None) == md.MD_ERR_STATE
    assert lib.md_verlet_step(h, 7, C.byref(a), None) == md.MD_ERR_ARG
    assert lib.md_energy(h, None, None, None) == md.MD_ERR_ARG
    assert lib.md_workspace_bind(h, None, 0, None) == md.MD_ERR_ARG
    assert lib.md_strerror(md.MD_ERR_STATE) == b"no workspace bound"
    lib.md_system_destroy(h)


def test_product_path_has_no_oracle_dependency():
    """The package and its sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1507_07068_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "orc_" not in txt, fn


def test_library_exports_nothing_but_the_boundary(lib):
    """Internal helpers stay hidden: the defined dynamic text symbols are the declared ones."""
    import shutil
    import subprocess
    if not shutil.which("nm"):
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--defined-only", md.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    text = sorted(l.split()[-1] for l in out.splitlines() if len(l.split()) == 3 and l.split()[1] == "T")
    assert text == sorted(declared_functions())
