"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host symbolic analysis matches the oracle's bit for bit."""
import os
import re

import numpy as np
import pytest

import paper_2609_31477_amd as mf
from oracle import sym as osym
from tests.test_oracle_sym import graph_csr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "mf.h")).read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(mf_\w+)\s*\(", hdr, flags=re.M))
    assert declared == set(mf.EXPORTS)
    L = mf.lib()
    for name in declared:
        assert hasattr(L, name), name


def assert_same(view, S):
    assert view.spec_version == 1
    assert np.array_equal(view.perm, S.perm)
    assert np.array_equal(view.front_ptr, S.front_ptr)
    assert np.array_equal(view.front_parent, S.front_parent)
    assert np.array_equal(view.rows_ptr, S.rows_ptr)
    assert np.array_equal(view.rows, S.rows)
    assert np.array_equal(view.var_etree, S.var_etree)


@pytest.mark.parametrize("seed", range(12))
def test_symbolic_bit_exact_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 41))
    m = int(rng.integers(0, 3 * n + 1))
    e = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(m, 2))]
    rp, ci = graph_csr(n, e)
    nr = int(rng.integers(0, min(3, n) + 1))
    root = rng.permutation(n)[:nr].tolist()
    leaf = int(rng.choice([1, 2, 4, 8]))
    v = mf.Symbolic(n, rp, ci, root, leaf_max=leaf).export()
    assert_same(v, osym.analyze(n, rp, ci, root, leaf_max=leaf))


def test_symbolic_worked_example():
    rp, ci = graph_csr(7, [(i, i + 1) for i in range(6)])
    v = mf.Symbolic(7, rp, ci, [], leaf_max=2).export()
    assert v.perm.tolist() == [0, 2, 1, 4, 6, 5, 3]
    assert v.front_parent.tolist() == [2, 2, 6, 5, 5, 6, -1]


@pytest.mark.parametrize("nx,ny,seed,leaf", [(16, 8, 0, 64), (32, 16, 3, 16), (64, 32, 0, 64)])
def test_symbolic_bit_exact_jacobian(nx, ny, seed, leaf):
    from vivjac import build_2d
    s = build_2d(nx, ny, seed)
    sy = mf.Symbolic(s.n, s.rowptr, s.colind, s.root, leaf_max=leaf)
    v = sy.export()
    S = osym.analyze(s.n, s.rowptr, s.colind, s.root, leaf_max=leaf)
    assert_same(v, S)
    npiv = np.diff(S.front_ptr).astype(float)
    m = np.diff(S.rows_ptr).astype(float)
    assert v.nominal_nnz_lu == pytest.approx(float((2 * m * npiv - npiv ** 2).sum()))


def test_symbolic_unsorted_duplicates():
    # unsorted columns and duplicate entries give the same analysis as the clean pattern
    rp, ci = graph_csr(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)])
    v1 = mf.Symbolic(6, rp, ci, [], leaf_max=1).export()
    rp2, ci2 = graph_csr(6, [(0, 1), (0, 1), (2, 3), (1, 2), (4, 5), (3, 4), (2, 1)])
    v2 = mf.Symbolic(6, rp2, ci2, [], leaf_max=1).export()
    assert np.array_equal(v1.perm, v2.perm) and np.array_equal(v1.rows, v2.rows)


def test_analyze_errors():
    rp, ci = graph_csr(3, [(0, 1)])
    with pytest.raises(mf.MFError) as e:
        mf.Symbolic(3, rp, ci, [3])
    assert e.value.status == mf.MF_ERR_ARG
    with pytest.raises(mf.MFError):
        mf.Symbolic(3, rp, np.array([7], dtype=np.int32))
    with pytest.raises(mf.MFError):
        mf.Symbolic(3, rp, ci, [1, 1])
    bad = rp.copy()
    bad[1] = 5
    with pytest.raises(mf.MFError):
        mf.Symbolic(3, bad, ci, [])


def test_empty_pattern():
    v = mf.Symbolic(0, np.zeros(1, np.int64), np.zeros(0, np.int32), []).export()
    assert v.nfronts == 0 and v.perm.size == 0


def test_footprint_positive(config0):
    s = config0
    sy = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    assert sy.footprint_bytes("fp64") > sy.footprint_bytes("fp32") > 0


@pytest.mark.slow
def test_symbolic_bit_exact_256x128():
    """The benchmark's own pattern (256x128 cells, n = 540,606): the library's
    analysis equals the oracle's bit for bit, at the size where it is timed."""
    from vivjac import build_2d
    s = build_2d(256, 128, 1)
    v = mf.Symbolic(s.n, s.rowptr, s.colind, s.root).export()
    S = osym.analyze(s.n, s.rowptr, s.colind, s.root)
    assert v.nfronts == S.nfronts
    assert_same(v, S)


def test_level_task_lists_count_equals_fill(tmp_path):
    """The per-level tile work lists are counted exactly before they are written
    into a fixed buffer (pinned host memory in the driver): a C++ check over random
    levels that the count equals the fill and that a short buffer is detected
    without a write past its end."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "test_tasks")
    src = os.path.join(ROOT, "tests", "csrc", "test_tasks.cpp")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", src, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("OK")


def test_sweep_work_list_protocol(tmp_path):
    """The persistent sweeps' work-list protocol, emulated on the CPU over random
    front forests and random interleavings of 1..64 work-groups: tickets,
    per-front counts and waits as in the kernels; no deadlock, every task runs
    once, and only after the tasks whose results it reads."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "test_sweep_protocol")
    src = os.path.join(ROOT, "tests", "csrc", "test_sweep_protocol.cpp")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", src, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("OK")


def test_ale_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "ale.h")).read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(ale_\w+)\s*\(", hdr, flags=re.M))
    assert declared == {"ale_create", "ale_residual", "ale_jacobian", "ale_device_bytes", "ale_release"}
    L = mf.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_ale_create_rejects_missing_coupling_and_bad_indices():
    """The set-up checks run on the host before anything touches a device: a
    pattern without a coupling of the element terms, and out-of-range numbers."""
    from paper_2609_31477_amd.ale import Assembly
    from vivjac.ale2d import build_ale_2d
    p = build_ale_2d(16, 8, 0)
    # drop one (u, x) coupling from the pattern
    r = int(p.u_dof[p.tri[40, 3], 0])           # an interior edge node's u_x row
    assert r >= 0
    lo, hi = int(p.rowptr[r]), int(p.rowptr[r + 1])
    cols = p.colind[lo:hi]
    drop = lo + int(np.flatnonzero(cols >= p.blocks["x"][0])[0])
    p.colind = np.delete(p.colind, drop)
    p.rowptr = p.rowptr.copy()
    p.rowptr[r + 1:] -= 1
    with pytest.raises(mf.MFError) as e:
        Assembly(p)
    assert e.value.status == mf.MF_ERR_PATTERN and "not in the pattern" in str(e.value)
    q = build_ale_2d(16, 8, 0)
    q.tri = q.tri.copy()
    q.tri[3, 2] = q.u_dof.shape[0] + 5
    with pytest.raises(mf.MFError) as e:
        Assembly(q)
    assert e.value.status == mf.MF_ERR_ARG and "tri" in str(e.value)


def test_factor_rejects_bad_options_before_any_device_call():
    """Option checks run on the host before the device is touched, so a bad
    refinement mode or precision is an argument error with no handle made."""
    import ctypes
    rp, ci = graph_csr(4, [(0, 1), (1, 2), (2, 3)])
    S = mf.Symbolic(4, rp, ci, [])
    L = mf.lib()
    for field, value in (("refine", 4), ("refine", 9), ("prec", 7), ("pivot_u", 2.0)):
        o = mf.mf_options()
        L.mf_default_options(ctypes.byref(o))
        setattr(o, field, value)
        h = ctypes.c_void_p()
        st = L.mf_factor(S._h, ctypes.c_void_p(64), ctypes.byref(o), None, ctypes.byref(h))
        assert st == mf.MF_ERR_ARG, (field, value)
        assert h.value is None
        assert field.split("_")[0] in L.mf_last_error().decode() or "precision" in L.mf_last_error().decode()
