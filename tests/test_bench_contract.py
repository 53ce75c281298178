"""Host-side parts of bench.py's output contract (no GPU needed).

* More than one GPU is refused with a message and exit status 2.
* roofline.traffic comes from the committed counter summary only while the
  kernel's sources hash to the value recorded beside the counters; a kernel
  with no recorded line, or sources that no longer match, gives None.
* The algorithmic flop count of one weight set follows its stated terms.
"""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def _digest(sources):
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, "paper_1912_06441_amd", "csrc", src), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _recorded(kernel):
    lines = []
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if name.endswith(".md"):
            with open(os.path.join(ROOT, "profiles", name)) as fh:
                lines += [ln.split() for ln in fh if ln.startswith("TRAFFIC " + kernel + " ")]
    return lines


@pytest.mark.parametrize("kernel,sources", [
    ("weights64_k8", ["weights.hip", "weights_common.hpp", "basis.hpp"]),
    ("weights64f_k8", ["weights_split.hip", "weights_common.hpp", "basis.hpp"]),
    ("apply_f64", ["apply.hip", "stencil_rows.hpp"]),
])
def test_traffic_follows_the_source_hash(kernel, sources):
    rec = _recorded(kernel)
    assert rec, "no counter line for %s" % kernel
    got = bench.measured_traffic(kernel, sources)
    match = [r for r in rec if r[2] == "src=" + _digest(sources)]
    if match:
        assert got == float(match[0][3].split("=")[1]) and got > 0
    else:
        assert got is None
    # a different set of sources (so a different hash) never borrows the line
    assert bench.measured_traffic(kernel, sources + ["burgers.hip"]) is None


def test_unknown_kernel_has_no_traffic():
    assert bench.measured_traffic("no_such_kernel", ["apply.hip"]) is None


def test_weight_flops_terms():
    # basis 10Np, assembly 2Np^2, LU 2p^3/3, (1 + it) x [solve 2 nd p^2 + weights 2 N p nd + residual 2 N p nd]
    N, p, nd = 60, 44, 3
    assert bench.weight_flops(N, p, nd, 0) == pytest.approx(10 * N * p + 2 * N * p * p + 2 * p ** 3 / 3
                                                            + 2 * nd * p * p + 4 * N * p * nd)
    step = bench.weight_flops(N, p, nd, 1) - bench.weight_flops(N, p, nd, 0)
    assert step == pytest.approx(2 * nd * p * p + 4 * N * p * nd)


def test_cpu_model_reports_processor_count():
    name, nproc = bench.cpu_model()
    assert isinstance(name, str) and nproc >= 1


def test_factor_flops_are_the_first_pass_of_weight_flops():
    # the factor kernel: basis 10Np, assembly 2Np^2, LU 2p^3/3, first solve 2 nd p^2; the rest of
    # weight_flops (weights and residual, and every refinement sweep) is the refine kernel's
    N, p, nd = 60, 44, 3
    assert bench.factor_flops(N, p, nd) == pytest.approx(10 * N * p + 2 * N * p * p + 2 * p ** 3 / 3 + 2 * nd * p * p)
    assert bench.weight_flops(N, p, nd, 0) - bench.factor_flops(N, p, nd) == pytest.approx(4 * N * p * nd)
