"""The C ABI as a C program sees it: tests/c/abi_smoke.c is compiled as C99
against include/ppr.h with gcc and linked to libppr.so.  Without a GPU the
program must get PPR_ERR_DEVICE from ppr_graph_create (exit 2); on a GPU it
must reproduce the Figure 1 values (exit 0)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2101_03652_amd")


def _build(tmp_path):
    exe = str(tmp_path / "abi_smoke")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c", "abi_smoke.c"), "-o", exe,
                           "-L", LIBDIR, "-lppr", f"-Wl,-rpath,{LIBDIR}", "-lm"])
    return exe


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_header_compiles_as_c99_and_links(tmp_path):
    exe = _build(tmp_path)
    if _has_gpu():
        pytest.skip("a GPU is present: the gpu-marked test runs the program")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 2, res.stdout + res.stderr


@pytest.mark.gpu
def test_c_program_reproduces_figure1(tmp_path):
    exe = _build(tmp_path)
    print("[gpu] C ABI program", flush=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
