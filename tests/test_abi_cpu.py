"""The C-ABI library loads on a CPU-only machine, exports every symbol the
public header declares, and its host-only validation rejects bad parameters.
No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2005_04642_amd import lbm, workloads as Wk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chromo_lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[A-Za-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load_library()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(lbm.EXPORTED) == names


def good():
    return lbm.make_params(64, 64, "f32", **Wk.base_params(Lambda=10.0))


def test_validate_accepts_workload_parameters():
    for storage in ("f32", "f64", "f16", "bf16"):
        for cfg in (Wk.config_static_drop(), Wk.config_layered_channel()):
            p = lbm.make_params(cfg["nx"], cfg["ny"], storage, **cfg["params"])
            assert lbm.lbm_validate_params(p)[0] == lbm.LBM_OK


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("storage", 7), ("walls_y", 2), ("rho0_B", 0.0), ("alpha_R", 1.0),
    ("alpha_B", 0.3), ("nu_R", 0.0), ("lambda6", 2.0), ("lambda7", 0.0), ("eps_n", 0.0),
    ("ghost_eq", 3), ("flags", 64), ("sigma", float("nan")),
])
def test_validate_rejects(field, value):
    p = good()
    setattr(p, field, value)
    code, msg = lbm.lbm_validate_params(p)
    assert code == lbm.LBM_EINVAL and msg


def test_validate_rejects_bad_stencil_and_huge_and_wall_height():
    p = good()
    p.stencil[2] = 2
    assert lbm.lbm_validate_params(p)[0] == lbm.LBM_EINVAL
    p = good()
    p.nx, p.ny = 40000, 40000          # more than 2^30 sites
    assert lbm.lbm_validate_params(p)[0] == lbm.LBM_EINVAL
    p = good()
    p.nx, p.ny = 16, 70000             # more rows than the grid's y dimension holds
    assert lbm.lbm_validate_params(p)[0] == lbm.LBM_EINVAL
    p = lbm.make_params(30_000_000, 2, "f64", **Wk.base_params(Lambda=10.0))  # one row of 4.3 GB
    assert lbm.lbm_validate_params(p)[0] == lbm.LBM_EINVAL
    p = good()
    p.walls_y, p.ny = 1, 2
    assert lbm.lbm_validate_params(p)[0] == lbm.LBM_EINVAL


def test_population_buffers_past_4_gib():
    """The step addresses each lattice row through a buffer resource of its own,
    so a whole population buffer may exceed 4 GiB (8192^2 FP32: 4.8 GB; 20000^2
    FP32: 28.8 GB) in every format.  A solid-site mask addresses the whole buffer
    through one resource (below 4 GiB).  The adjoint's workspace rows are
    addressed with 64-bit offsets: every accepted lattice has one."""
    for storage in ("f32", "f16", "bf16", "f64"):
        for n in (8192, 10240, 20000):
            p = lbm.make_params(n, n, storage, **Wk.base_params(Lambda=10.0))
            assert lbm.lbm_validate_params(p)[0] == lbm.LBM_OK, (storage, n)
    big = lbm.make_params(8192, 8192, "f32", **Wk.base_params(Lambda=10.0))
    assert lbm.lbm_solid_workspace_bytes(big) == 0
    assert lbm.lbm_adjoint_workspace_bytes(big) > 0
    small = lbm.make_params(7680, 7680, "f32", **Wk.base_params(Lambda=10.0))
    assert lbm.lbm_solid_workspace_bytes(small) > 0
    huge = lbm.make_params(11000, 11000, "f32", **Wk.base_params(Lambda=10.0))
    assert lbm.lbm_adjoint_workspace_bytes(huge) >= 39 * 4 * 11000 * 11000
    largest = lbm.make_params(32768, 32768, "f32", **Wk.base_params(Lambda=10.0))
    assert lbm.lbm_adjoint_workspace_bytes(largest) >= 39 * 4 * 32768 * 32768


def test_sizes():
    p = good()
    assert lbm.lbm_pops_elems(p) == 18 * 64 * 64
    assert lbm.lbm_pops_bytes(p) == 4 * 18 * 64 * 64
    for storage, words, nbytes in (("f64", 18, 8), ("f16", 10, 4), ("bf16", 10, 4)):
        q = lbm.make_params(64, 32, storage, **Wk.base_params(Lambda=10.0))
        assert lbm.lbm_pops_elems(q) == words * 64 * 32
        assert lbm.lbm_pops_bytes(q) == nbytes * words * 64 * 32
    assert lbm.lbm_workspace_bytes(p) > 0
    p.nx = 0
    assert lbm.lbm_workspace_bytes(p) == 0


def test_init_argument_errors_before_any_gpu_call():
    lib = lbm.load_library()
    p = good()
    h = ctypes.c_void_p()
    code = lib.lbm_init(ctypes.byref(p), None, None, None, None, None, 0, None, ctypes.byref(h))
    assert code == lbm.LBM_EINVAL and h.value is None
    code = lib.lbm_step(None, 1, None, None)
    assert code == lbm.LBM_EINVAL


def test_adjoint_availability_and_argument_errors():
    """The adjoint exists for F64/F32 storage, periodic or walled; its
    workspace size is 0 for the 16-bit formats, and NULL arguments fail before
    any GPU call."""
    lib = lbm.load_library()
    prm = Wk.base_params(Lambda=10.0)
    for storage, walls, ok in (("f32", False, True), ("f64", False, True), ("f16", False, False),
                               ("bf16", False, False), ("f32", True, True), ("f64", True, True),
                               ("f16", True, False)):
        p = lbm.make_params(64, 48, storage, **dict(prm, walls=walls))
        n = lbm.lbm_adjoint_workspace_bytes(p)
        assert (n > 0) == ok, (storage, walls)
        if ok:
            elem = 8 if storage == "f64" else 4
            assert n >= 39 * 64 * 48 * elem
    assert lib.lbm_adjoint_step(None, None, None, None, None, 0, None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_rhoN_adjoint(None, None, None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_init_adjoint(None, None, None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_set_pops(None, None, None) == lbm.LBM_EINVAL


def test_batch_validation_and_layout():
    prm = Wk.base_params(Lambda=10.0)
    ps = [lbm.make_params(n, m, "f32", **prm) for n, m in ((64, 64), (5, 7), (300, 20))]
    total = lbm.lbm_batch_pops_bytes(ps)
    offs = lbm.lbm_batch_offsets(ps)
    assert offs[0] == 0 and all(o % 256 == 0 for o in offs)
    assert offs[1] >= 72 * 64 * 64 and offs[2] - offs[1] >= 72 * 5 * 7
    assert total >= offs[2] + 72 * 300 * 20
    assert lbm.lbm_batch_workspace_bytes(ps) > 0
    walls = [lbm.make_params(64, 64, "f32", **dict(prm, walls=True)),
             lbm.make_params(40, 30, "f32", **dict(prm, walls=True))]
    assert lbm.lbm_batch_pops_bytes(walls) > 0                      # all walled: allowed
    assert lbm.lbm_batch_pops_bytes([ps[0], walls[0]]) == 0          # periodic and walled mixed
    fast = [lbm.make_params(64, 64, "f32", **dict(prm, walls=True, stencil=(3, 1, 3, 1)))]
    assert lbm.lbm_batch_pops_bytes(fast) > 0                        # walled: 3333, 3131, 1111
    odd = [lbm.make_params(64, 64, "f32", **dict(prm, walls=True, stencil=(1, 3, 1, 3)))]
    assert lbm.lbm_batch_pops_bytes(odd) == 0
    mixed = [ps[0], lbm.make_params(64, 64, "f64", **prm)]
    assert lbm.lbm_batch_pops_bytes(mixed) == 0
    radii = [ps[0], lbm.make_params(64, 64, "f32", **dict(prm, stencil=(1, 1, 1, 1)))]
    assert lbm.lbm_batch_pops_bytes(radii) == 0


def test_solid_mask_availability_and_argument_errors():
    """Masks of solid sites exist for every storage format without walls (14
    field planes of workspace); NULL arguments fail before any GPU call."""
    lib = lbm.load_library()
    prm = Wk.base_params(Lambda=10.0)
    for storage, walls, ok in (("f32", False, True), ("f64", False, True), ("f16", False, True),
                               ("bf16", False, True), ("f32", True, False)):
        p = lbm.make_params(64, 48, storage, **dict(prm, walls=walls))
        n = lbm.lbm_solid_workspace_bytes(p)
        assert (n > 0) == ok, (storage, walls)
        if ok:
            assert n >= 14 * 64 * 48 * (8 if storage == "f64" else 4) and n % 256 == 0
    assert lib.lbm_set_solid(None, None, None, 0, None) == lbm.LBM_EINVAL
    assert lib.lbm_batch_set_solid(None, 0, None, None, 0, None) == lbm.LBM_EINVAL
    assert lib.lbm_batch_set_force(None, 0, None, None) == lbm.LBM_EINVAL


def test_partition_stream_and_cu_budget_argument_checks():
    """Checked before any device call: CU ranges in multiples of 8, a handle
    for the CU budget."""
    for first, count in ((3, 8), (0, 0), (-8, 8), (8, 12)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_partition_stream(first, count)
        assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_cu_budget(None, 0, 0)
    assert e.value.code == lbm.LBM_EINVAL


def test_trajectory_entry_point_argument_checks():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step_into(None, None, [], None)
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_adjoint_steps(None, [], None, None, None, 0, None, None, None)
    assert e.value.code == lbm.LBM_EINVAL


def test_plain_c_program_uses_the_abi(tmp_path):
    """The header is plain C (C99, -Wall -Wextra -Werror) and a C program
    linked against the library gets the documented results of the host-side
    entry points (tests/c_consumer.c; no GPU needed)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.join(root, "paper_2005_04642_amd")
    exe = str(tmp_path / "c_consumer")
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(root, "include"), "-I", "/opt/rocm/include",
           os.path.join(root, "tests", "c_consumer.c"), "-o", exe,
           "-L", libdir, "-lchromo_lbm", "-Wl,-rpath," + libdir]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failed checks" in r.stdout
