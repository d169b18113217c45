"""Host-side checks of the C ABI: the library loads, exports every declared symbol,
validates arguments and sizes workspaces.  No GPU compute is launched here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fld.h")

fld = pytest.importorskip("paper_2104_03968_amd", reason="libfld.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fld_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(fld.LIB_PATH)
    names = declared_functions()
    assert "fld_step" in names and "fld_exchange" in names and "fld_plan_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(fld.EXPORTED) <= set(names) | {"fld_last_error"}


def test_strerror_and_version():
    assert fld.fld_version() >= 100
    for code in range(-9, 2):
        assert isinstance(fld.fld_strerror(code), str) and fld.fld_strerror(code)
    assert fld.fld_strerror(12345) == "unknown status"


def test_defaults():
    o = fld.fld_opts_default()
    assert o.c == 1.0 and o.rtol == 1e-10 and o.nu1 == 2 and o.nu2 == 2 and o.max_cycles == 50
    assert o.limiter == fld.FLD_LIMITER_LP and o.precision == fld.FLD_PREC_FP64
    assert o.fmg == 1 and o.fmg_depths == -1 and o.coarse_op == fld.FLD_COARSE_REDISCRETISED
    assert o.nu_coarse == 3 and o.tile_rows_up == 0
    assert fld.fld_opts_default(coarse_op="galerkin").coarse_op == fld.FLD_COARSE_GALERKIN
    g = fld.fld_gas_default()
    assert g.max_halley == 100 and g.root_rtol == pytest.approx(8.88e-16, rel=1e-2)


@pytest.mark.parametrize("n,ok", [((64, 64), True), ((3, 5), True), ((1, 8), False), ((0, 8), False),
                                  ((8, 8, 8), True), ((8, 8, 1), False)])
def test_plan_create_validates_grids(n, ok):
    g = fld.make_grid(n)
    if ok:
        h = fld.fld_plan_create([g], fld.fld_opts_default())
        assert fld.fld_plan_workspace_bytes(h) > 0
        fld.fld_plan_destroy(h)
    else:
        with pytest.raises(fld.FLDError) as e:
            fld.fld_plan_create([g], fld.fld_opts_default())
        assert e.value.code == fld.FLD_ERR_INVALID_ARG


@pytest.mark.parametrize("kw,code", [
    (dict(rtol=0.0), -1), (dict(rtol=2.0), -1), (dict(c=-1.0), -1), (dict(limiter=7), -1),
    (dict(precision=3), -1), (dict(max_cycles=0), -1), (dict(nu1=0, nu2=0), -1),
    (dict(bc=[5, 0, 0, 0, 0, 0]), fld.FLD_ERR_UNSUPPORTED), (dict(bc=[-1, 0, 0, 0, 0, 0]), -1),
    (dict(bc=[3, 0, 0, 0, 0, 0]), -1), (dict(bc=[0, 0, 0, 3, 0, 0]), -1),
    (dict(bc=[2, 0, 0, 0, 0, 0], bc_value=[-1.0, 0, 0, 0, 0, 0]), -1),
    (dict(bc=[0, 2, 0, 0, 0, 0], bc_value=[0, float("inf"), 0, 0, 0, 0]), -1),
    (dict(bc=[1, 0, 0, 0, 0, 0], bc_grad=[float("nan"), 0, 0, 0, 0, 0]), -1),
    (dict(fmg=2), -1), (dict(fmg=-1), -1), (dict(coarse_op=2), -1), (dict(coarse_op=-1), -1),
    (dict(fmg_depths=-2), -1), (dict(fmg_depths=65), -1), (dict(nu_coarse=-1), -1), (dict(nu_coarse=17), -1)])
def test_plan_create_validates_options(kw, code):
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default(**kw))
    assert e.value.code == code


@pytest.mark.parametrize("kw,ok", [
    (dict(tile_rows=4), True), (dict(tile_rows=8), True), (dict(tile_rows=32), True), (dict(tile_rows=12), False),
    (dict(tile_wide=1), True), (dict(tile_wide=2), False), (dict(max_blocks=512), True),
    (dict(max_blocks=-1), False), (dict(autotune=1), True), (dict(autotune=2), True),
    (dict(autotune=3), False), (dict(autotune=1, tile_rows=16), False),
    (dict(autotune=1, max_blocks=1024), False),
    # an FP64 128-wide, 32-row tile with the nu = 2 halo needs more than the 160 KB of LDS
    (dict(tile_wide=1, tile_rows=32), False), (dict(tile_wide=1, tile_rows=32, precision=1), True),
    (dict(tile_wide=1, tile_rows=32, nu1=1, nu2=1, nu_coarse=1), True),
    # ... and the default three coarse sweeps' halo does not fit a 32-row coarse tile
    (dict(tile_wide=1, tile_rows=32, nu1=1, nu2=1), False),
    (dict(tile_wide=1, tile_rows=32, fused=0), True), (dict(tile_depth=16), True),
    (dict(tile_depth=64), True), (dict(tile_depth=24), False), (dict(autotune=1, tile_depth=32), False),
    (dict(fused3_levels=2), True), (dict(fused3_levels=-1), False), (dict(autotune=1, fused3_levels=1), False),
    (dict(fused=2), True), (dict(fused=3), True), (dict(fused=4), False), (dict(fused=-1), False),
    (dict(tile_rows_coarse=4), True), (dict(tile_rows_coarse=12), False),
    (dict(autotune=1, tile_rows_coarse=8), False), (dict(tile_wide=1, tile_rows_coarse=32), False),
    (dict(tile_rows_up=16), True), (dict(tile_rows_up=6), False), (dict(autotune=1, tile_rows_up=8), False),
    (dict(tile_wide=1, tile_rows_up=32), True), (dict(tile_wide=1, tile_rows=16, tile_rows_up=4), True),
    # the coarse levels' tile carries the nu_coarse halo; a count the fused kernels do not
    # take sends the plan to the per-colour sweeps, which have no tile to fit
    (dict(tile_wide=1, tile_rows_coarse=32, nu_coarse=1), True),
    (dict(tile_wide=1, tile_rows=32, nu1=1, nu2=1, nu_coarse=2), False),
    (dict(tile_wide=1, tile_rows=32, nu_coarse=4), True), (dict(nu_coarse=16), True)])
def test_launch_shape_options(kw, ok):
    g = fld.make_grid((256, 256))
    if ok:
        fld.fld_plan_destroy(fld.fld_plan_create([g], fld.fld_opts_default(**kw)))
    else:
        with pytest.raises(fld.FLDError) as e:
            fld.fld_plan_create([g], fld.fld_opts_default(**kw))
        assert e.value.code == fld.FLD_ERR_INVALID_ARG


def test_unknown_option_name_is_an_error():
    with pytest.raises(TypeError):
        fld.fld_opts_default(tile_row=8)


def test_tile_shape_does_not_change_the_workspace():
    g = [fld.make_grid((300, 196)), fld.make_grid((1024, 1024))]
    sizes = set()
    for kw in (dict(), dict(tile_rows=8), dict(tile_wide=1, tile_rows=16), dict(max_blocks=64), dict(autotune=1)):
        h = fld.fld_plan_create(g, fld.fld_opts_default(**kw))
        sizes.add(fld.fld_plan_workspace_bytes(h))
        fld.fld_plan_destroy(h)
    assert len(sizes) == 1


def test_bad_h_rejected():
    g = fld.make_grid((16, 16), (0.1, -0.1))
    with pytest.raises(fld.FLDError):
        fld.fld_plan_create([g], fld.fld_opts_default())


def test_hierarchy_levels_and_workspace_scaling():
    cases = {(1024, 1024): 10, (480, 480): 6, (96, 96): 6, (3, 5): 1, (64, 64, 64): 6, (176, 176, 176): 5}
    for n, nl in cases.items():
        h = fld.fld_plan_create([fld.make_grid(n)], fld.fld_opts_default())
        assert fld.fld_plan_levels(h, 0) == nl, n
        fld.fld_plan_destroy(h)
    # workspace, 2D FP64: level 0 holds w_x, w_y, X, B0, R (+ P0, P1, Q, Z under CG), and
    # the coarse levels x, b, w_x, w_y on N/3 cells in total
    N = 1024 * 1024
    sizes = {}
    for kw in (dict(fused=0), dict(krylov=0, fused=0), dict(precision=1, fused=0), dict()):
        h = fld.fld_plan_create([fld.make_grid((1024, 1024))], fld.fld_opts_default(**kw))
        sizes[tuple(kw.items())] = fld.fld_plan_workspace_bytes(h) / N
        fld.fld_plan_destroy(h)
    cg64, mg64 = sizes[(("fused", 0),)], sizes[(("krylov", 0), ("fused", 0))]
    assert 8 * 9 + 32 / 3 <= cg64 <= 8 * 9 + 32 / 3 + 1
    assert 8 * 5 + 32 / 3 <= mg64 <= 8 * 5 + 32 / 3 + 1
    # fused 2D levels keep the down pass's output apart: one more array on every level
    # that has a coarser one (~4/3 N cells)
    assert cg64 + 8 * 4 / 3 - 1 <= sizes[()] <= cg64 + 8 * 4 / 3 + 1
    cg32 = sizes[(("precision", 1), ("fused", 0))]
    # FP64 w_x, w_y, X, B0, R, P0, P1, Q at level 0, FP64 coarse weights, FP32 hierarchy
    assert 8 * 8 + 16 / 3 + 16 * 4 / 3 <= cg32 <= 8 * 8 + 16 / 3 + 16 * 4 / 3 + 1


def test_batched_plan_workspace_is_sum_of_parts():
    grids = [fld.make_grid((n, n)) for n in (64, 96, 128)]
    hb = fld.fld_plan_create(grids, fld.fld_opts_default())
    parts = 0
    for g in grids:
        h = fld.fld_plan_create([g], fld.fld_opts_default())
        parts += fld.fld_plan_workspace_bytes(h)
        fld.fld_plan_destroy(h)
    assert fld.fld_plan_workspace_bytes(hb) <= parts
    assert [fld.fld_plan_levels(hb, i) for i in range(3)] == [6, 6, 7]   # coarsest 2, 3, 2
    fld.fld_plan_destroy(hb)


def test_calls_before_bind_fail_cleanly():
    h = fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default())
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_level_view(h, 0, 0)
    assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
    rc, _ = fld.fld_step(h, [1], [1], [1], [1e-3], stream=0, check=False)
    assert rc == fld.FLD_ERR_NO_WORKSPACE
    with pytest.raises(fld.FLDError):
        fld.fld_plan_levels(h, 5)
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_tuning(h)
    assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_cycle_bytes(h, fld.FLD_CYCLE_ITERATION)
    assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
    fld.fld_plan_destroy(h)


def test_bind_rejects_small_or_null_workspace():
    h = fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default(use_graph=0))
    nb = fld.fld_plan_workspace_bytes(h)
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_bind_workspace(h, 0, nb)
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_bind_workspace(h, 4096, nb - 1)
    assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
    fld.fld_plan_destroy(h)


def test_server_defaults_and_argument_checks():
    o = fld.fld_server_opts_default()
    assert o.max_slots == 64 and o.precision == fld.FLD_PREC_MIXED and o.rtol == 1e-10
    assert o.cycles_per_round == 2
    with pytest.raises(fld.FLDError) as e:
        fld.fld_server_create(o, 0, 1 << 20)
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    with pytest.raises(fld.FLDError) as e:
        fld.fld_server_create(o, 4096 + 8, 1 << 20)          # misaligned arena
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    bad = fld.fld_server_opts_default(max_slots=0)
    with pytest.raises(fld.FLDError):
        fld.fld_server_create(bad, 4096, 1 << 20)


def test_library_binds_to_torchs_hip_runtime(tmp_path):
    """The package imports torch before loading libfld.so, so the library's HIP symbols
    (the kernel registration at load time included) resolve to torch's runtime rather
    than a second HIP runtime in the same process, whatever the caller imported first."""
    import subprocess
    import sys
    out = tmp_path / "ld"
    env = dict(os.environ, LD_DEBUG="bindings", LD_DEBUG_OUTPUT=str(out))
    code = ("import sys; sys.path.insert(0, %r); import paper_2104_03968_amd as f; "
            "f.fld_opts_default()" % ROOT)
    subprocess.run([sys.executable, "-c", code], env=env, check=True, timeout=300)
    import torch
    torch_lib = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), "lib"))
    lines = []
    for p in tmp_path.iterdir():
        lines += [ln for ln in p.read_text(errors="replace").splitlines()
                  if "libfld.so" in ln and "__hipRegisterFatBinary'" in ln]
    assert lines, "no binding of __hipRegisterFatBinary recorded"
    for ln in lines:
        target = ln.split(" to ", 1)[1].split(" [")[0]
        assert os.path.realpath(target).startswith(torch_lib), ln


def test_moments_need_a_bound_workspace():
    h = fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default())
    with pytest.raises(fld.FLDError) as e:
        fld.fld_radiation_moments(h, [1], [1], [{}], stream=0)
    assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
    fld.fld_plan_destroy(h)


def test_imex_scratch_size_and_argument_checks():
    shapes = [(48, 64), (10, 12, 14)]
    h = fld.fld_plan_create([fld.make_grid(tuple(reversed(s))) for s in shapes], fld.fld_opts_default())
    per = [((64 * 48 * 8 + 255) // 256) * 256, ((14 * 12 * 10 * 8 + 255) // 256) * 256]
    assert fld.fld_imex_scratch_bytes(h, fld.FLD_IMEX_EULER) == 2 * sum(per)
    assert fld.fld_imex_scratch_bytes(h, fld.FLD_IMEX_MIDPOINT) == 4 * sum(per)
    with pytest.raises(fld.FLDError) as e:
        fld.fld_imex_scratch_bytes(h, 7)
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    gas = fld.fld_gas_default(c=1.0)
    one = [4096, 8192]
    # before bind; then a gas c that differs from the plan's c
    rc, _ = fld.fld_imex_step(h, one, one, one, one, [1e-3] * 2, gas, fld.FLD_IMEX_EULER, 4096, 1 << 30,
                              stream=0, check=False)
    assert rc == fld.FLD_ERR_NO_WORKSPACE
    rc, _ = fld.fld_imex_step(h, one, one, one, one, [1e-3] * 2, fld.fld_gas_default(c=2.0),
                              fld.FLD_IMEX_EULER, 4096, 1 << 30, stream=0, check=False)
    assert rc in (fld.FLD_ERR_NO_WORKSPACE, fld.FLD_ERR_INVALID_ARG)
    fld.fld_plan_destroy(h)


def test_fixed_gradient_boundaries_are_accepted():
    o = fld.fld_opts_default(bc=[1, 1, 0, 0, 0, 0], bc_grad=[0.5, -2.0, 0, 0, 0, 0])
    assert list(o.bc)[:2] == [fld.FLD_BC_FIXED_GRADIENT] * 2 and list(o.bc_grad)[:2] == [0.5, -2.0]
    h = fld.fld_plan_create([fld.make_grid((16, 16))], o)
    fld.fld_plan_destroy(h)



def test_fmg_and_galerkin_plans():
    """The full-multigrid start adds only work-lists to the descriptor region; the
    Galerkin coarse operator changes no layout."""
    grids = [fld.make_grid((64, 96)), fld.make_grid((16, 24, 20)), fld.make_grid((37, 50))]
    sizes = {}
    for kw in (dict(fmg=0), dict(fmg=1), dict(fmg=0, coarse_op="galerkin"), dict(fmg=1, precision=1, krylov=0)):
        h = fld.fld_plan_create(grids, fld.fld_opts_default(**kw))
        sizes[tuple(sorted(kw.items()))] = fld.fld_plan_workspace_bytes(h)
        assert [fld.fld_plan_levels(h, i) for i in range(3)] == [6, 3, 1]
        fld.fld_plan_destroy(h)
    base = sizes[(("fmg", 0),)]
    assert sizes[(("coarse_op", "galerkin"), ("fmg", 0))] == base
    assert 0 <= sizes[(("fmg", 1),)] - base <= 64 * 1024


def test_dirichlet_plans_add_one_coupling_array_per_level():
    grids = [fld.make_grid((64, 48)), fld.make_grid((16, 16, 8))]
    sizes = {}
    for prec in (0, 1):
        for bc in ([0] * 6, [2, 0, 0, 2, 0, 0]):
            h = fld.fld_plan_create(grids, fld.fld_opts_default(precision=prec, bc=bc, bc_value=[1.0] * 6))
            sizes[(prec, bc[0])] = fld.fld_plan_workspace_bytes(h)
            fld.fld_plan_destroy(h)
    # per-colour sweeps (no xs arrays of the fused kernels) with 8 B per cell and level of
    # couplings (+4 B in mixed precision): compare against zero-flux plans that also sweep
    # per colour
    for prec in (0, 1):
        h = fld.fld_plan_create(grids, fld.fld_opts_default(precision=prec, fused=0))
        base = fld.fld_plan_workspace_bytes(h)
        fld.fld_plan_destroy(h)
        n = 64 * 48 + 32 * 24 + 16 * 12 + 8 * 6 + 4 * 3 + 16 * 16 * 8 + 8 * 8 * 4 + 4 * 4 * 2
        extra = sizes[(prec, 2)] - base
        assert (8 + 4 * prec) * n <= extra <= (8 + 4 * prec) * n + 2 * 256 * 8 + 4096


def test_continuous_faces_need_plain_vcycles():
    """Continuous faces make the operator unsymmetric: CG plans are refused."""
    bc = [fld.FLD_BC_CONTINUOUS, fld.FLD_BC_ZERO_FLUX, 0, 0, 0, 0]
    with pytest.raises(fld.FLDError) as e:
        fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default(bc=bc))
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    h = fld.fld_plan_create([fld.make_grid((16, 16))], fld.fld_opts_default(bc=bc, krylov=0))
    fld.fld_plan_destroy(h)


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets (a field
    added on one side only would shift the rest silently)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    names = ["fld_grid", "fld_opts", "fld_stats", "fld_gas", "fld_level_view", "fld_moments_out", "fld_tuning",
             "fld_server_opts", "fld_request", "fld_result", "fld_server_info"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fld.h"', 'int main(void) {']
    for n in names:
        lines.append(f'    printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in getattr(fld, n)._fields_:
            lines.append(f'    printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ['    return 0;', '}']
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "sizes"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        n, f, v = line.split()
        cls = getattr(fld, n)
        want = C.sizeof(cls) if f == "size" else getattr(cls, f).offset
        assert int(v) == want, (n, f, int(v), want)
