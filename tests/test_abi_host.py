"""Host-side checks of the C ABI: the library loads, exports every entry
point that include/pimpc.h declares, and rejects bad input during host
validation (which runs before any HIP call, so no GPU is needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pimpc.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pimpc_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ["pimpc_setup", "pimpc_linearize", "pimpc_solve", "pimpc_solve_batch", "pimpc_backward"]:
        assert n in names
    assert set(names) == set(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
        assert ctypes.cast(getattr(L, n), ctypes.c_void_p).value


def test_version_and_defaults():
    assert P.pimpc_version() == 2
    o = P.pimpc_default_options()
    assert o.rho == 1.0 and o.max_iter == 200 and o.precision == P.PIMPC_FP32
    assert o.eta == pytest.approx(0.999) and o.check_every == 1


def _setup_code(problems, **kw):
    o = P.pimpc_default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    try:
        ctx, _ = P.pimpc_setup(problems, o)
    except P.PimpcError as e:
        return e.code, e.msg
    P.pimpc_destroy(ctx)
    return 0, ""


@pytest.mark.parametrize("field,value", [("rho", 0.0), ("rho", -1.0), ("rho", float("inf")),
                                         ("max_iter", 0), ("check_every", 0), ("precision", 7),
                                         ("accel", 3), ("warm_start", 2), ("ckpt_every", -1),
                                         ("eps", float("nan")), ("family", 3), ("family", -1)])
def test_bad_options_rejected(field, value):
    code, msg = _setup_code([W.plain_fp64_problem(0)], **{field: value})
    assert code == P.PIMPC_E_ARG, (field, value, code, msg)


def test_instance_count_beyond_the_setup_grid_is_refused():
    """More than 65535 instances: PIMPC_E_DIM from host validation (the setup
    kernels give each instance one row of their grid)."""
    p = W.plain_fp64_problem(0).copy(N=1)
    code, msg = _setup_code([p] * 65536)
    assert code == P.PIMPC_E_DIM and "65535" in msg


def test_bad_problem_data_rejected():
    p = W.plain_fp64_problem(0)
    q = p.copy(xmin=p.xmin.copy())
    q.xmin[2] = 5.0  # xmin > xmax
    assert _setup_code([q])[0] == P.PIMPC_E_ARG
    q = p.copy(A=p.A.copy())
    q.A[1, 1] = np.nan
    assert _setup_code([q])[0] == P.PIMPC_E_NONFINITE
    q = p.copy(Q=p.Q.copy())
    q.Q[0, 0] = -1.0
    assert _setup_code([q])[0] == P.PIMPC_E_NOT_PSD
    q = p.copy(R=p.R.copy())
    q.R[0, 1] = 0.3  # not symmetric
    code, msg = _setup_code([q])
    assert code == P.PIMPC_E_NOT_PSD and "symmetric" in msg
    q = p.copy(N=0)
    assert _setup_code([q])[0] == P.PIMPC_E_DIM


def test_bad_constraint_sets_rejected():
    p = W.plain_fp64_problem(0)
    assert _setup_code([p.copy(uset=("soc",))])[0] not in (P.PIMPC_E_ARG, P.PIMPC_E_DIM)
    q = W.Problem(**{**p.__dict__, "uset": ("halfspace", np.zeros(3), 1.0)})
    code, msg = _setup_code([q])
    assert code == P.PIMPC_E_ARG and "normal" in msg
    code, msg = _setup_code([p.copy(uset=("l1ball", -0.1))])
    assert code == P.PIMPC_E_ARG and "radius" in msg
    code, msg = _setup_code([p.copy(xset=("l1ball", float("nan")))])
    assert code == P.PIMPC_E_NONFINITE
    # a cone needs two entries
    one = W.cartpole_problem(N=16, K=5).copy(uset=("soc",))
    assert _setup_code([one])[0] == P.PIMPC_E_DIM
    # non-box sets: no tape
    code, msg = _setup_code([p.copy(uset=("soc",))], ckpt_every=20)
    assert code == P.PIMPC_E_UNSUPPORTED and "box" in msg


def test_bad_rate_weight_rejected():
    p = W.plain_fp64_problem(0)
    Wd = 0.1 * np.eye(3)
    Wd[0, 2] = 0.05  # not symmetric
    code, msg = _setup_code([p.copy(Wdu=Wd)])
    assert code == P.PIMPC_E_NOT_PSD and "Wdu" in msg and "symmetric" in msg
    code, msg = _setup_code([p.copy(Wdu=np.diag([0.1, -0.2, 0.1]))])
    assert code == P.PIMPC_E_NOT_PSD and "Wdu" in msg
    Wd = 0.1 * np.eye(3)
    Wd[1, 1] = np.nan
    assert _setup_code([p.copy(Wdu=Wd)])[0] == P.PIMPC_E_NONFINITE


def test_unsupported_requests_are_reported():
    # the taped forward differentiates plain ADMM
    code, msg = _setup_code([W.plain_fp64_problem(0)], accel=1, ckpt_every=20)
    assert code == P.PIMPC_E_UNSUPPORTED and "accel" in msg
    # ... over exactly max_iter iterations, with either kind of tape
    for ck in (1, 20):
        code, msg = _setup_code([W.plain_fp64_problem(0)], eps=1e-4, ckpt_every=ck)
        assert code == P.PIMPC_E_UNSUPPORTED and "eps" in msg


def test_shapes_without_a_kernel_are_reported():
    """Valid problems no compiled kernel serves: a stage wider than the widest
    long-horizon class, and a long horizon in FP64 (the long-horizon family
    iterates in FP32)."""
    rng = np.random.default_rng(0)
    nx, nu = 40, 10
    wide = W.Problem(nx=nx, nu=nu, N=600, A=np.eye(nx) * 0.9, B=rng.standard_normal((nx, nu)) * 0.1,
                     Q=np.eye(nx), R=np.eye(nu), xmin=-np.ones(nx), xmax=np.ones(nx), umin=-np.ones(nu),
                     umax=np.ones(nu), x0=np.zeros(nx), u_prev=np.zeros(nu), K=10)
    code, msg = _setup_code([wide])
    assert code == P.PIMPC_E_UNSUPPORTED and "no compiled kernel" in msg
    lh = W.long_horizon_problem(0, N=600, K=10)
    code, msg = _setup_code([lh], precision=P.PIMPC_FP64)
    assert code == P.PIMPC_E_UNSUPPORTED and "fp64" in msg
    # a long time-varying horizon with stages wider than 24 + 12
    rng2 = np.random.default_rng(1)
    nx2, nu2, N2 = 30, 14, 600
    tvw = W.Problem(nx=nx2, nu=nu2, N=N2, A=np.broadcast_to(np.eye(nx2) * 0.9, (N2, nx2, nx2)).copy(),
                    B=rng2.standard_normal((N2, nx2, nu2)) * 0.1, Q=np.eye(nx2), R=np.eye(nu2),
                    xmin=-np.ones(nx2), xmax=np.ones(nx2), umin=-np.ones(nu2), umax=np.ones(nu2),
                    x0=np.zeros(nx2), u_prev=np.zeros(nu2), K=10)
    code, msg = _setup_code([tvw])
    assert code == P.PIMPC_E_UNSUPPORTED and "no compiled kernel" in msg
    # FP64 lane classes stop at nx + nu = 13 (padded), where the stage still fits a lane's registers
    big = W.random_batch(64, base_seed=1000, K=10)
    big = [p for p in big if p.nx + p.nu > 13][0]
    code, msg = _setup_code([big], precision=P.PIMPC_FP64)
    assert code == P.PIMPC_E_UNSUPPORTED and "no compiled kernel" in msg


@pytest.mark.parametrize("eta", [0.0, -0.5, 1.5, float("nan")])
def test_bad_restart_threshold_rejected(eta):
    assert _setup_code([W.plain_fp64_problem(0)], accel=1, eta=eta)[0] == P.PIMPC_E_ARG


def test_error_text_available_without_context():
    code, msg = _setup_code([W.plain_fp64_problem(0)], rho=-2.0)
    assert code == P.PIMPC_E_ARG and "rho" in msg
    assert b"rho" in P.lib().pimpc_last_error(None)


def test_requested_family_that_cannot_serve_is_unsupported():
    """options.family forces a kernel family; setup refuses, before any HIP
    call, an instance that family cannot serve."""
    long = W.long_horizon_problem(0, N=600, K=10)  # nx = 24: no lane-family class
    code, msg = _setup_code([long], family=P.PIMPC_FAMILY_LANE)
    assert code == P.PIMPC_E_UNSUPPORTED and "lane-family" in msg
    small = W.plain_fp64_problem(0)
    code, _ = _setup_code([small], family=P.PIMPC_FAMILY_ROW, precision=P.PIMPC_FP64)  # row: FP32 only
    assert code == P.PIMPC_E_UNSUPPORTED


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of pimpc_problem, pimpc_options and pimpc_info have
    the C compiler's field offsets and sizes (a C program built against
    include/pimpc.h prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pimpc_problem": P.pimpc_problem, "pimpc_options": P.pimpc_options, "pimpc_info": P.pimpc_info}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pimpc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for name, cls in structs.items():
        assert int(got[f"{name} size"]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_output_form_validation():
    """The output form of eqn. (1) is folded on the host: a bounded output
    that mixes states is unsupported, bounds that empty a state box and a
    non-PSD output weight are rejected, all before any HIP call."""
    p = W.afti16_problem(N=5)
    mixed = p.copy(C=np.array([[0.0, 1.0, 0.0, 0.5], [0.0, 0.0, 0.0, 1.0]]))
    code, msg = _setup_code([mixed])
    assert code == P.PIMPC_E_UNSUPPORTED and "mixes" in msg
    empty = p.copy(xmin=np.array([-np.inf, 0.6, -np.inf, -np.inf]))  # y_1 <= 0.5 and x_2 >= 0.6
    code, msg = _setup_code([empty])
    assert code == P.PIMPC_E_ARG and "empty" in msg
    bad = p.copy(Wy=np.diag([100.0, -1.0]))
    code, msg = _setup_code([bad])
    assert code == P.PIMPC_E_NOT_PSD and "Wy" in msg
    nanr = p.copy(ry=np.array([0.0, np.nan]))
    assert _setup_code([nanr])[0] == P.PIMPC_E_NONFINITE
    soc = p.copy(xset=("soc",))
    code, msg = _setup_code([soc])
    assert code == P.PIMPC_E_UNSUPPORTED and "box" in msg
