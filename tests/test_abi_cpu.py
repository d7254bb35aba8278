"""CPU checks of the C ABI: the library loads and exports every function declared in
include/dpm.h; host-side validation rejects bad arguments without touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:dpm_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_abi():
    names = _declared()
    for must in ["aux_solve", "aux_solve_batched", "dpm_build_boundary_matrix", "dpm_step",
                 "dpm_gamma_points", "dpm_last_error", "dpm_workspace_size", "dpm_cfl_scan",
                 "dpm_bep_rebuild", "dpm_run"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1811_03557_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_host_validation_without_device():
    from paper_1811_03557_amd import _lib
    lib = _lib.load()
    o = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0)
    nb = C.c_size_t(0)
    bad = [_lib.Grid(6, 0.1, 1.0, 0.0),      # n + 1 not a power of two
           _lib.Grid(7, -0.1, 1.0, 0.0),     # h <= 0
           _lib.Grid(7, 0.1, -1.0, 0.0),     # sigma < 0
           _lib.Grid(7, 0.1, float("nan"), 0.0)]
    for g in bad:
        assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(o), C.byref(nb)) == _lib.DPM_EINVAL
        assert lib.dpm_last_error()
    g = _lib.Grid(255, 3.0 / 256, 1.0, 0.0)
    assert lib.dpm_workspace_size(C.byref(g), 0, C.byref(o), C.byref(nb)) == _lib.DPM_EINVAL
    # FP32 I/O only without refinement
    o2 = _lib.Opts(_lib.DPM_FP32, 0, 1e-10, 2, 0, None, 0)
    assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(o2), C.byref(nb)) == _lib.DPM_EINVAL
    # plain FP64 needs no volume workspace in the per-axis layout (the library's choice at
    # 255), and the separator planes of a launch in the split layout (its choice at 511: 31
    # planes of 511^2 reals per right-hand side); FP32 + FP64 I/O needs one FP32 volume per chunk
    assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(o), C.byref(nb)) == _lib.DPM_OK
    assert nb.value < 4096
    osp = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0, _lib.DPM_SWEEPS_SPLIT)
    assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(osp), C.byref(nb)) == _lib.DPM_OK
    assert 15 * 255**2 * 8 <= nb.value < 15 * 255**2 * 8 + 4096
    assert lib.dpm_workspace_size(C.byref(g), 64, C.byref(osp), C.byref(nb)) == _lib.DPM_OK
    assert 2 * 15 * 255**2 * 8 <= nb.value < 2 * 15 * 255**2 * 8 + 8192
    g511 = _lib.Grid(511, 3.0 / 512, 1.0, 0.0)
    assert lib.dpm_workspace_size(C.byref(g511), 1, C.byref(o), C.byref(nb)) == _lib.DPM_OK
    assert 31 * 511**2 * 8 <= nb.value < 31 * 511**2 * 8 + 4096
    oax = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0, _lib.DPM_SWEEPS_AXIS)
    assert lib.dpm_workspace_size(C.byref(g511), 1, C.byref(oax), C.byref(nb)) == _lib.DPM_OK
    assert nb.value < 4096
    # the split layout: plain solves at n = 255, 511 only
    g127s = _lib.Grid(127, 3.0 / 128, 1.0, 0.0)
    assert lib.dpm_workspace_size(C.byref(g127s), 1, C.byref(osp), C.byref(nb)) == _lib.DPM_EINVAL
    assert "DPM_SWEEPS_SPLIT" in lib.dpm_last_error().decode()
    for bad in (_lib.Opts(_lib.DPM_FP64, 1, 1e-10, 2, 0, None, 0, _lib.DPM_SWEEPS_SPLIT),
                _lib.Opts(_lib.DPM_FP32, 1, 1e-10, 2, 0, None, 0, _lib.DPM_SWEEPS_SPLIT),
                _lib.Opts(_lib.DPM_BF16X3, 1, 1e-10, 2, 0, None, 0, _lib.DPM_SWEEPS_SPLIT)):
        assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(bad), C.byref(nb)) == _lib.DPM_EINVAL
    of32 = _lib.Opts(_lib.DPM_FP32, 0, 1e-10, 0, 0, None, 0, _lib.DPM_SWEEPS_SPLIT)
    assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(of32), C.byref(nb)) == _lib.DPM_OK
    assert nb.value >= 15 * 255**2 * 4
    o3 = _lib.Opts(_lib.DPM_FP32, 1, 1e-10, 2, 1, None, 0)
    assert lib.dpm_workspace_size(C.byref(g), 4, C.byref(o3), C.byref(nb)) == _lib.DPM_OK
    assert nb.value >= 255**3 * 4
    # N + 1 not a power of two (N = 36, a mesh of the paper): FP64 takes it (Bluestein's sweeps,
    # without refinement), FP32 does not and names the forms that do
    g36 = _lib.Grid(36, 3.0 / 37, 1.0, 0.0)
    assert lib.dpm_workspace_size(C.byref(g36), 1, C.byref(o), C.byref(nb)) == _lib.DPM_OK
    o36r = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 2, 0, None, 0)
    assert lib.dpm_workspace_size(C.byref(g36), 1, C.byref(o36r), C.byref(nb)) == _lib.DPM_EINVAL
    o36f = _lib.Opts(_lib.DPM_FP32, 1, 1e-10, 2, 0, None, 0)
    assert lib.dpm_workspace_size(C.byref(g36), 1, C.byref(o36f), C.byref(nb)) == _lib.DPM_EINVAL
    msg = lib.dpm_last_error().decode()
    assert "DPM_FP64_GEMM" in msg and "Bluestein" in msg
    g700 = _lib.Grid(700, 3.0 / 701, 1.0, 0.0)  # beyond both the Bluestein and the dense sizes
    assert lib.dpm_workspace_size(C.byref(g700), 1, C.byref(o), C.byref(nb)) == _lib.DPM_EINVAL
    # sweep layouts: the plane sweeps exist for FFT-form FP64/FP32 at n <= 127 only
    g127 = _lib.Grid(127, 3.0 / 128, 1.0, 0.0)
    op = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0, _lib.DPM_SWEEPS_PLANE)
    assert lib.dpm_workspace_size(C.byref(g127), 1, C.byref(op), C.byref(nb)) == _lib.DPM_OK
    assert lib.dpm_workspace_size(C.byref(g), 1, C.byref(op), C.byref(nb)) == _lib.DPM_EINVAL
    assert "DPM_SWEEPS_PLANE" in lib.dpm_last_error().decode()
    ob = _lib.Opts(_lib.DPM_BF16X3, 1, 1e-10, 2, 0, None, 0, _lib.DPM_SWEEPS_PLANE)
    assert lib.dpm_workspace_size(C.byref(g127), 1, C.byref(ob), C.byref(nb)) == _lib.DPM_EINVAL
    ox = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0, 7)
    assert lib.dpm_workspace_size(C.byref(g127), 1, C.byref(ox), C.byref(nb)) == _lib.DPM_EINVAL
    og = _lib.Opts(_lib.DPM_FP64_GEMM, 1, 1e-10, 0, 0, None, 0)
    assert lib.dpm_workspace_size(C.byref(g36), 1, C.byref(og), C.byref(nb)) == _lib.DPM_OK
    g600 = _lib.Grid(600, 3.0 / 601, 1.0, 0.0)
    assert lib.dpm_workspace_size(C.byref(g600), 1, C.byref(og), C.byref(nb)) == _lib.DPM_EINVAL
    # null pointers are rejected before any launch
    assert lib.aux_solve(C.byref(g), None, None, C.byref(o), None, None) == _lib.DPM_EINVAL
    # misaligned volumes and bad per-right-hand-side sigmas are rejected before any launch
    fake = C.c_void_p(0x10000)
    odd = C.c_void_p(0x10004)
    assert lib.aux_solve(C.byref(g), odd, fake, C.byref(o), None, None) == _lib.DPM_EINVAL
    assert "aligned" in lib.dpm_last_error().decode()
    for bad_sig in ([1.0, -1.0], [float("nan"), 1.0], [1.0, float("inf")]):
        sg = (C.c_double * 2)(*bad_sig)
        assert lib.aux_solve_batched_sigma(C.byref(g), 2, sg, fake, C.c_void_p(0x90000000),
                                           C.byref(o), None, None) == _lib.DPM_EINVAL
        assert "sigma" in lib.dpm_last_error().decode()
    # the adaptive loop's entry points reject a missing handle before any launch
    prm = _lib.RunParams(1.0, 1.0, float("inf"), 10)
    assert lib.dpm_run(None, C.byref(prm), fake, odd, C.byref(o), None, None, None, None) == _lib.DPM_EINVAL
    assert lib.dpm_bep_rebuild(None, 1.0, None, 0, None) == _lib.DPM_EINVAL
    assert lib.dpm_run_workspace_size(None, C.byref(o), None) == _lib.DPM_EINVAL
    assert lib.dpm_bep_rebuild_workspace_size(None, None) == _lib.DPM_EINVAL
    # dpm_step: the outputs must be two buffers, every volume 8-byte aligned (checked before the
    # handle is read, so a stand-in handle pointer is never dereferenced)
    h = C.c_void_p(0x70000000)
    a, b2 = C.c_void_p(0x80000000), C.c_void_p(0x80100000)
    st = lib.dpm_step(h, 0.1, 1.0, a, b2, b2, b2, C.byref(o), None, None)
    assert st == _lib.DPM_EINVAL and "different buffers" in lib.dpm_last_error().decode()
    st = lib.dpm_step(h, 0.1, 1.0, a, b2, C.c_void_p(0x80200004), b2, C.byref(o), None, None)
    assert st == _lib.DPM_EINVAL and "aligned" in lib.dpm_last_error().decode()
    assert lib.dpm_cfl_scan(None, fake, fake, fake, None) == _lib.DPM_EINVAL


def test_dd_validation_without_device():
    """The domain-decomposition entry points reject bad radii, degrees, meshes and handles before
    any launch."""
    from paper_1811_03557_amd import _lib
    lib = _lib.load()
    g1 = _lib.Grid(15, 0.09375, 1000.0, -0.75 + 0.09375)
    g2 = _lib.Grid(31, 0.09375, 1000.0, -1.5 + 0.09375)
    o = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0)
    out = C.c_void_p(0)

    def build(**kw):
        p = dict(grid1=g1, grid2=g2, center=(C.c_double * 3)(0, 0, 0), r_z=0.5, r_gamma=1.0,
                 r_split=0.75, m_gamma=2, beta=1, m_z=2)
        p.update(kw)
        prm = _lib.DDParams(**p)
        return lib.dpm_dd_build(C.byref(prm), C.byref(o), None, C.byref(out), None)

    for kw, word in [({"r_split": 0.4}, "radii"), ({"r_gamma": 0.7}, "radii"),
                     ({"r_z": 0.0}, "radii"), ({"beta": 2}, "beta"), ({"m_z": -1}, "m_gamma"),
                     ({"m_gamma": 600}, "columns"),
                     ({"grid2": _lib.Grid(31, 0.09375, 999.0, -1.5 + 0.09375)}, "sigma"),
                     ({"grid1": _lib.Grid(700, 0.09375, 1000.0, -0.75)}, "n + 1")]:
        assert build(**kw) == _lib.DPM_EINVAL, kw
        assert word in lib.dpm_last_error().decode(), (kw, lib.dpm_last_error())
    assert out.value is None
    fake = C.c_void_p(256)
    vols = (C.c_void_p * 4)(256, 512, 768, 1024)
    assert lib.dpm_dd_step(None, 1e-3, 1.0, vols, vols, C.byref(o), None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_masks(None, 0, fake, fake, None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_gauss_state(None, 0, 1.0, 1.0, (C.c_double * 3)(0, 0, 0), fake, None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_info(None, None, None, None, None, None, None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_lsq_info(None, None, None, None) == _lib.DPM_EINVAL
    m = C.c_int32(0)
    assert lib.dpm_dd_lsq_method(None, C.byref(m)) == _lib.DPM_EINVAL
    assert lib.dpm_bep_lsq_method(None, C.byref(m)) == _lib.DPM_EINVAL
    # Case 2: Z must meet Gamma
    g1b = _lib.Grid(15, 0.09375, 1000.0, -0.75 + 0.09375)

    def build2(**kw):
        p = dict(grid1=g1b, grid2=g2, origin1=(C.c_double * 3)(0, 0, 0.75),
                 origin2=(C.c_double * 3)(0, 0, 0), r_gamma=1.0, q_z=1.0, r_z=0.5, eps_layers=2.0,
                 m_gamma=4, beta=0, m_z=2)
        p.update(kw)
        prm = _lib.DD2Params(**p)
        return lib.dpm_dd2_build(C.byref(prm), C.byref(o), None, C.byref(out), None)

    for kw, word in [({"q_z": 2.0}, "meets"), ({"q_z": 0.3}, "meets"), ({"eps_layers": 0.0}, "eps"),
                     ({"beta": 3}, "beta"), ({"origin1": (C.c_double * 3)(0, float("nan"), 0)}, "origins"),
                     ({"rcond": -1e-7}, "rcond"), ({"rcond": 1.0}, "rcond"),
                     ({"rcond": 1e-7, "m_gamma": 700}, "640 columns")]:
        assert build2(**kw) == _lib.DPM_EINVAL, kw
        assert word in lib.dpm_last_error().decode(), (kw, lib.dpm_last_error())
    prm = _lib.RunParams(1.0, 1.0, float("inf"), 10)
    assert lib.dpm_dd_rebuild(None, 1.0, None, 0, None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_run_workspace_size(None, C.byref(o), None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_rebuild_workspace_size(None, None) == _lib.DPM_EINVAL
    assert lib.dpm_dd_run(None, C.byref(prm), vols, C.byref(o), None, None, None, None) == _lib.DPM_EINVAL


def test_diagnostics_workspace_constant_and_validation():
    """The binding's scratch size equals the header's define; a missing or short scratch and a
    missing handle are rejected before any launch."""
    from paper_1811_03557_amd import _lib
    src = open(os.path.join(ROOT, "include", "dpm.h")).read()
    m = re.search(r"#define DPM_DIAG_WORKSPACE_BYTES \(\(size_t\)(\d+)\)", src)
    assert m and int(m.group(1)) == _lib.DPM_DIAG_WORKSPACE_BYTES
    lib = _lib.load()
    fake = C.c_void_p(256)
    assert lib.dpm_diagnostics(fake, fake, fake, fake, None, 0, None) == _lib.DPM_EINVAL
    assert "workspace" in lib.dpm_last_error().decode()
    assert lib.dpm_diagnostics(fake, fake, fake, fake, fake, 100, None) == _lib.DPM_EINVAL
    assert lib.dpm_diagnostics(None, fake, fake, fake, fake, 1 << 20, None) == _lib.DPM_EINVAL
    vols = (C.c_void_p * 4)(256, 512, 768, 1024)
    assert lib.dpm_dd_diagnostics(None, vols, fake, fake, 1 << 20, None) == _lib.DPM_EINVAL


def test_autotune_validation_without_device():
    """dpm_autotune checks its arguments on the host before any device work; with nothing tuned,
    dpm_rhs_chunk reports the default width (2 FP64 volumes at 255^3, about 256 MB)."""
    from paper_1811_03557_amd import _lib
    lib = _lib.load()
    lib.dpm_autotune_reset()
    g = _lib.Grid(255, 3.0 / 256, 1.0, 0.0)
    o = _lib.Opts(_lib.DPM_FP64, 1, 1e-10, 0, 0, None, 0)
    w = C.c_int32(0)
    assert lib.dpm_rhs_chunk(C.byref(g), 64, C.byref(o), C.byref(w)) == _lib.DPM_OK and w.value == 2
    nc = _lib.DPM_TUNE_MAX_CANDIDATES
    widths, lays, zc, ms = (C.c_int32 * nc)(), (C.c_int32 * nc)(), (C.c_int32 * nc)(), (C.c_double * nc)()
    cnt, best, bl, bz = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
    args = (widths, lays, zc, ms, C.byref(cnt), C.byref(best), C.byref(bl), C.byref(bz))
    for nrhs, reps in ((0, 3), (4, 0), (4, 101)):
        assert lib.dpm_autotune(C.byref(g), nrhs, C.byref(o), None, None, reps, None, *args) == _lib.DPM_EINVAL
        assert lib.dpm_last_error()
    assert lib.dpm_autotune(C.byref(g), 4, C.byref(o), None, None, 3, None, *args) == _lib.DPM_EINVAL
    assert b"NULL" in lib.dpm_last_error()
    bad = _lib.Grid(6, 0.1, 1.0, 0.0)
    assert lib.dpm_autotune(C.byref(bad), 4, C.byref(o), None, None, 3, None, *args) == _lib.DPM_EINVAL
