"""Host logic of the search plan (plan.hpp, built here with g++ for the host):
the threshold sample each call shape gets, and the plan's invariants.  The
sample grows past the minimum only where the candidates it saves cost more than
its columns: short reduced-precision rows, not the long FP32 rows."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F32, BF16, FP8 = 0, 1, 2


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_probe")
    subprocess.run(["g++", "-std=c++17", "-O1", "-w", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "paper_1309_5478_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "plan_probe.cpp"), "-o", exe], check=True)

    def run(m, n, d, k, graph, prec, env=None):
        e = dict(os.environ)
        e.pop("KNN_SAMPLE_COLS", None)
        e.update(env or {})
        out = subprocess.run([exe, str(m), str(n), str(d), str(k), str(int(graph)), str(prec)], env=e,
                             capture_output=True, text=True, check=True).stdout.split()
        return tuple(int(x) for x in out)
    return run


def test_measured_shapes(probe):
    # k-NNG 262144 x 1024, k = 32, FP32: the minimum sample (S k' >= 2N) stands
    S, r, cap, kk = probe(262144, 262144, 1024, 32, True, F32)
    assert (S, kk, cap) == (4096, 128, 2304)
    # the same in BF16: twice the sample (768 -> 512 candidates expected)
    assert probe(262144, 262144, 1024, 32, True, BF16)[0] == 8192
    # k-NNG 2^20 x 256, k = 64: 16384 columns in every precision
    for prec in (BF16, FP8, F32):
        S, r, cap, kk = probe(1 << 20, 1 << 20, 256, 64, True, prec)
        assert (S, kk) == (16384, 256)
        assert (r + 1) * ((1 << 20) - 1) / S <= 1100   # expected candidates per row
    # the override
    assert probe(1 << 20, 1 << 20, 256, 64, True, BF16, {"KNN_SAMPLE_COLS": "8192"})[0] == 8192


@pytest.mark.parametrize("prec", [F32, BF16, FP8])
def test_plan_invariants(probe, prec):
    for n in (5000, 40037, 262144, 1 << 20, 3 << 20):
        for d in (64, 256, 1024):
            for k in (1, 16, 64, 256, 1024):
                S, r, cap, kk = probe(4096, n, d, k, False, prec)
                assert kk == min(4 * k, 1024, n)
                assert S <= 16384 and (S == n or S & (S - 1) == 0)
                assert S >= 2048 or S == n
                assert 0 <= r < S and r < 1024
                assert cap <= 4096 and cap % 64 == 0
                assert cap >= min(kk + 64, 4096)
                if S < n:
                    expected = (r + 1) * n / S
                    assert expected >= kk                 # the threshold aims above the k'-th
                    assert S * kk >= 2 * n or S == 16384      # the minimum sample
