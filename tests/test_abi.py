"""CPU checks of the C ABI: the library loads, exports every declared entry point,
and validates descriptors on the host (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def T():
    import paper_1009_2768_amd as T
    from paper_1009_2768_amd import build
    if build.stale():
        build.build()
    T.load()
    return T


def declared_functions():
    src = open(os.path.join(ROOT, "include", "trmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trmc_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree(T):
    from paper_1009_2768_amd import _abi
    assert declared_functions() == sorted(_abi.EXPORTS)


def test_library_exports_every_declared_symbol(T):
    lib = ctypes.CDLL(T._abi.lib_path())
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version_and_strerror(T):
    L = T.load()
    assert L.trmc_abi_version() == 2
    for code in (0, -22, -12, -28, -5, -75):
        assert len(L.trmc_strerror(code)) > 0


def test_struct_sizes_match_header(T, tmp_path):
    """sizeof of the ABI structs as compiled by the host C compiler."""
    from paper_1009_2768_amd import _abi
    src = tmp_path / "s.c"
    src.write_text('#include <stdio.h>\n#include "trmc.h"\nint main(){printf("%zu %zu %zu\\n", sizeof(trmc_desc),'
                   ' sizeof(trmc_particles), sizeof(trmc_cell_moments));return 0;}\n')
    exe = tmp_path / "s"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    a, b, c = map(int, subprocess.check_output([str(exe)]).split())
    assert a == ctypes.sizeof(_abi.Desc)
    assert b == ctypes.sizeof(_abi.Particles)
    assert c == ctypes.sizeof(_abi.CellMoments)


def _ws(T, **kw):
    d = T.Instance(**kw).to_c()
    n = ctypes.c_size_t(0)
    return T.load().trmc_workspace_size(ctypes.byref(d), 1, ctypes.byref(n)), n.value


@pytest.mark.parametrize("bad", [
    dict(n_particles=0), dict(n_particles=100, geometry=3), dict(n_particles=100, precision=7),
    dict(n_particles=100, n_cells=2), dict(n_particles=100, geometry=2, n_cells=0),
    dict(n_particles=100, geometry=2, n_cells=100000), dict(n_particles=100, dt=0.0),
    dict(n_particles=100, eps=0.0), dict(n_particles=100, alpha=1.5), dict(n_particles=100, trunc=9),
    dict(n_particles=100, m_cap=0), dict(n_particles=100, m_cap=5000), dict(n_particles=100, m_init=70),
    dict(n_particles=100, trunc=2, delta1=0.02, delta2=0.01), dict(n_particles=100, particle_weight=-1.0),
    # tree-shape truncation: unknown definition, m_max 0, combined with the adaptive depth
    dict(n_particles=100, trunc=1, wb=3), dict(n_particles=100, trunc=1, wb=1, wb_mmax=0),
    dict(n_particles=100, trunc=2, wb=2, wb_mmax=5), dict(n_particles=100, trunc=3, wb=1, wb_mmax=5),
    dict(n_particles=100, trunc=4), dict(n_particles=100, trunc=3, delta1=0.02, delta2=0.01),
    # majorant raised level by level: unknown mode, with reuse, with tree-shape truncation
    dict(n_particles=100, majorant=2), dict(n_particles=100, trunc=3, majorant=1),
    dict(n_particles=100, trunc=1, wb=1, wb_mmax=2, majorant=1),
])
def test_invalid_descriptors_rejected(T, bad):
    rc, _ = _ws(T, **bad)
    assert rc == -22


@pytest.mark.parametrize("ok", [dict(n_particles=100, trunc=1, wb=1, wb_mmax=1),
                                dict(n_particles=100, trunc=0, wb=2, wb_mmax=64),
                                dict(n_particles=100, trunc=2, alpha=1.0, majorant=1)])
def test_tree_shape_truncation_descriptors_accepted(T, ok):
    rc, n = _ws(T, **ok)
    assert rc == 0 and n > 0


def test_workspace_size_grows_with_particles(T):
    rc1, a = _ws(T, n_particles=1000)
    rc2, b = _ws(T, n_particles=100000)
    rc3, c = _ws(T, n_particles=100000, precision=T.FP32_MIXED)
    assert rc1 == rc2 == rc3 == 0 and a < b and c < b


def test_struct_size_guard(T):
    d = T.Instance(n_particles=100).to_c()
    d.struct_size = 8
    n = ctypes.c_size_t(0)
    assert T.load().trmc_workspace_size(ctypes.byref(d), 1, ctypes.byref(n)) == -22


def test_no_cpu_fallback_without_gpu(T):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU visible")
    with pytest.raises(RuntimeError):
        T.Context([T.Instance(n_particles=10)], [{"vx": None, "vy": None, "vz": None}])
