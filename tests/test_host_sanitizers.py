"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the pass
planner over every size and cap, the tile order of the pass launches, the cost-diagonal pieces against the plain
definition of the cost, the L-BFGS driver on Rosenbrock and on
objectives that fail or stop, and the CPU oracle's routines on small instances.
Built with the host compilers only (no GPU code)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_13012_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
ROCM_INCLUDE = "/opt/rocm/include"
FLAGS = ["-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build_and_run(tmp_path, name, sources, extra):
    exe = str(tmp_path / name)
    cmd = ["g++", *FLAGS, *extra, "-I", CSRC, "-I", os.path.join(ROOT, "include"), *sources, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_planner_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "plan_check",
                         [os.path.join(HOST, "plan_check.cpp"), os.path.join(CSRC, "plan.cpp")],
                         ["-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE])
    assert "plans ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_tile_order_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "xcd_check", [os.path.join(HOST, "xcd_check.cpp")],
                         ["-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE])
    assert "tile order ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_cost_pieces_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "cost_pieces_check",
                         [os.path.join(HOST, "cost_pieces_check.cpp"), os.path.join(CSRC, "cost_terms.cpp")],
                         ["-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE])
    assert "cost pieces ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_lbfgs_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "lbfgs_check",
                         [os.path.join(HOST, "lbfgs_check.cpp"), os.path.join(CSRC, "lbfgs.cpp")], [])
    assert "lbfgs ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(HOST, "oracle_check.c"),
           os.path.join(ROOT, "oracle", "qaoa_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "oracle ok" in out.stdout
