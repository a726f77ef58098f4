"""The C-ABI library loads and exports every function include/tdslda.h
declares (no GPU needed: nothing here launches a kernel)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tdslda.h")).read()
    return sorted(set(re.findall(r"\b(tdslda_[a-z_0-9]+)\s*\(", txt)))


def test_header_functions_are_exported():
    from paper_2602_08982_amd import tdslda as T
    lib = T.load_library()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(T.EXPORTED)


def test_memory_plan_and_kernel_names():
    from paper_2602_08982_amd import tdslda as T
    b64 = T.memory_plan(T.lattice_3d(32), T.run_config(precision=T.FP64), 32768)
    b32 = T.memory_plan(T.lattice_3d(32), T.run_config(precision=T.FP32_MIXED), 32768)
    # 6 state-sized buffers dominate: 6 * 32768 states * 1 MiB (FP64)
    assert 6 * 32768 * 2 ** 20 < b64 < 6.3 * 32768 * 2 ** 20
    assert 0.45 < b32 / b64 < 0.55
    assert "lap2_full" in T.kernel_names()
    with pytest.raises(T.TdsldaError):
        T.memory_plan(T.lattice_3d(10), T.run_config(), 10)  # unsupported shape


def test_host_fft_templates(tmp_path):
    """The in-register DFT templates (compiled for the host) against direct
    sums: forward DFT, second derivative (full k^2), first derivative with
    the Nyquist bin zeroed, and the Parseval kinetic sum."""
    src = os.path.join(ROOT, "tests", "native", "fft_host_test.hip")
    exe = str(tmp_path / "fft_host_test")
    subprocess.run(["hipcc", "-O1", "-std=c++17", "--offload-arch=gfx950", "-o", exe, src], check=True,
                   capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
