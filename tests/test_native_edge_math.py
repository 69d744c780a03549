"""CPU check of the per-edge device math (host build of the same functions the
kernels call): the hand-written edge-flux VJP against central differences of
the edge flux, for both WENO powers and with/without the positivity fallback.
WENO eps = 1e-6 (with 1e-40 the nonlinear weights are not differentiable in
near-uniform data; see the adjoint tests)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "check_edge_math.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("native") / "check_edge_math")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", f"-I{ROOT}/include",
                    f"-I{ROOT}/paper_2102_12933_amd/csrc", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", SRC, "-o", out], check=True, capture_output=True)
    return out


@pytest.mark.parametrize("positivity,power,riemann,cons,uni,eps,tol", [
    (1, 1, 0, 0, 0, "1e-6", 1e-7), (0, 1, 0, 0, 0, "1e-6", 1e-7), (1, 2, 0, 0, 0, "1e-6", 1e-6),
    (1, 1, 1, 0, 0, "1e-6", 2e-5), (1, 1, 0, 0, 1, "1e-6", 1e-7),
    # conservative components have smoothness indicators nearer eps: the weights are stiffer and the
    # central differences' own truncation error grows (4e-7 at eps 1e-6, 2e-8 at 1e-4, 1e-9 at 1e-2)
    (1, 1, 0, 1, 0, "1e-4", 1e-7)])
def test_edge_vjp_matches_finite_differences(exe, positivity, power, riemann, cons, uni, eps, tol):
    r = subprocess.run([exe, str(tol), str(positivity), str(power), eps, str(riemann), str(cons), str(uni)],
                       capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
