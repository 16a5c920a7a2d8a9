"""Host-only checks of libdgmi.so (no GPU needed): every symbol declared in
include/dg.h is exported, configuration validation, and the host helpers
(Gauss nodes, OU driving update) agree with the independent oracle."""
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1602_09079_amd import dg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(dg.LIB_PATH):
        from paper_1602_09079_amd import build
        build.build()
    yield


def header_functions():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(dg.EXPORTS)


def test_every_declared_symbol_is_exported():
    L = dg.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_library_shares_torchs_hip_runtime():
    """Loaded first in a fresh process, before anything imports torch, the library still maps
    one HIP runtime: torch's, so that torch's streams and buffers are valid for it."""
    import subprocess
    import sys
    code = ("from paper_1602_09079_amd import dg\n"
            "dg.lib()\n"
            "print(len(dg.hip_runtimes()))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout


def test_nmodes():
    for k in range(5):
        assert dg.nmodes(k) == O.nmodes(k)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_gauss_nodes_match_oracle(n):
    np.testing.assert_allclose(dg.gauss_nodes(n), O.gauss_legendre(n)[0], atol=3e-16)


def test_gauss_nodes_rejects_out_of_range():
    for n in (0, 6, -1):
        with pytest.raises(dg.DGError):
            dg.gauss_nodes(n)


def test_ou_update_matches_oracle():
    nvec = synth.forcing_modes()
    th = synth.ou_stationary_start(1602, len(nvec))
    z = synth.ou_normals(1602, len(nvec), 3)
    tg, to = th.copy(), th.copy()
    for j in range(3):
        tg, ag = dg.ou_update(nvec, tg, z[j], 0.9, 1.0, 0.7, 1.0, 3.0)
        to, ao = O.ou_update(nvec, to, z[j], 0.9, 1.0, 0.7, 1.0, 3.0)
        np.testing.assert_allclose(tg, to, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(ag, ao, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kw,status", [
    (dict(k=-1, n=8), dg.DG_ERR_ARG),
    (dict(k=5, n=8), dg.DG_ERR_UNSUPPORTED),
    (dict(k=4, n=8, precision="bf16"), dg.DG_ERR_UNSUPPORTED),  # k = 4: FP64 and FP32 storage only
    (dict(k=4, n=8, precision="bf16x3"), dg.DG_ERR_UNSUPPORTED),
    (dict(k=1, n=(8, 1, 8)), dg.DG_ERR_ARG),
    (dict(k=1, n=8, box=(1.0, 0.0, 1.0)), dg.DG_ERR_ARG),
    (dict(k=1, n=8, gamma=1.0), dg.DG_ERR_ARG),
    (dict(k=1, n=8, cfl=0.0), dg.DG_ERR_ARG),
    (dict(k=1, n=8, cfl=1.5), dg.DG_ERR_ARG),
    (dict(k=1, n=8, precision=7), dg.DG_ERR_ARG),
    (dict(k=1, n=8, flags=128), dg.DG_ERR_ARG),
    (dict(k=2, n=8, flags=dg.DG_CLOSURE), dg.DG_ERR_UNSUPPORTED),
])
def test_config_validation(kw, status):
    assert dg.init_status(dg.make_config(**kw)) == status
    why = dg.lib().dg_error_string(None).decode()
    assert why.startswith("dg_init: ") and len(why) > len("dg_init: "), why  # the reason is kept


def test_mlp_host_helpers():
    shape = (140, 128, 128, 20)
    assert dg.mlp_nparams(shape) == O.mlp_nparams(*shape) == 37140
    assert dg.lib().dg_mlp_workspace_bytes(dg._shape_arr(shape), 4096) >= 4 * 4096 * (140 + 4 * 128 + 3 * 20)
    assert dg.mlp_nparams((0, 1, 1, 1)) == 0
    # invalid arguments are rejected before any device work
    assert dg.lib().dg_adam(10, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == dg.DG_ERR_ARG
    assert dg.lib().dg_column_stats(None, 10, 3, None, None, None, None, None, None) == dg.DG_ERR_ARG


def test_column_stats_noalloc_rejects_before_device_work():
    """The allocation-free column statistics reject NULL pointers and more columns than the static
    scratch holds (160) before any device call, with the reason in dg_error_string(NULL)."""
    L = dg.lib()
    fake = 4096  # non-NULL placeholders: the checks return before any pointer is used
    assert L.dg_column_stats_noalloc(None, 10, 3, fake, fake, fake, fake, None) == dg.DG_ERR_ARG
    assert "NULL" in L.dg_error_string(None).decode()
    assert L.dg_column_stats_noalloc(fake, 10, 161, fake, fake, fake, fake, None) == dg.DG_ERR_ARG
    assert "160" in L.dg_error_string(None).decode()
    assert L.dg_column_stats_noalloc(fake, 0, 3, fake, fake, fake, fake, None) == dg.DG_ERR_ARG
