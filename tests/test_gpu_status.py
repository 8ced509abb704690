"""Device-detected numeric problems reach the host: a non-finite Lanczos
coefficient (forced with a NaN weight on a graph built without the check)
makes slaq_graph_info return SLAQ_ERR_NUMERIC and sets the device status
word; non-finite coefficients handed to the Gauss-rule eigensolve (§3.1,
eq. "quadratic"; Algorithm 1's eigh) make it reach its sweep cap, which sets
SLAQ_STATUS_NO_CONVERGENCE.  Every kernel still exits normally: the
eigensolve's sweeps are bounded and NaN arithmetic does not trap."""
import numpy as np
import pytest
import torch

from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

pytestmark = pytest.mark.gpu


def test_nan_weight_without_check_reports_numeric():
    print("\n[gpu] status: NaN weight, Chung-Lu n=500, no CSR check", flush=True)
    S.device_status(clear=True)
    csr = inputs.chung_lu(500, 2000, 2.5, seed=3)
    rp, ci = S.to_device(csr)
    w = np.ones(csr.nnz, dtype=np.float32)
    w[10] = np.nan
    g = S.build_graph(rp, ci, torch.from_numpy(w).cuda(), check=False)
    S.lanczos(g, 8, 10, seed=1)
    torch.cuda.synchronize()
    with pytest.raises(S.SlaqError) as e:
        g.info()
    assert e.value.status == S.SLAQ_ERR_NUMERIC
    bits = S.device_status(clear=True)
    assert bits & S.SLAQ_STATUS_NONFINITE
    assert S.device_status(clear=True) == 0  # cleared by the previous call
    # the same graph with finite weights reports nothing
    g2 = S.build_graph(rp, ci)
    a, b, s = S.lanczos(g2, 8, 10, seed=1)
    S.ritz(a, b, s)
    g2.info()
    assert S.device_status(clear=True) == 0


def test_nonfinite_tridiagonal_reaches_the_sweep_cap():
    print("\n[gpu] status: NaN / Inf Lanczos coefficients into the eigensolves", flush=True)
    S.device_status(clear=True)
    nv, m = 5, 8
    alpha = torch.full((nv, m), 0.7, dtype=torch.float64, device="cuda")
    beta = torch.full((nv, m), 0.2, dtype=torch.float64, device="cuda")
    steps = torch.full((nv,), m, dtype=torch.int32, device="cuda")
    th, w2 = S.ritz(alpha, beta, steps)
    assert S.device_status(clear=True) == 0 and torch.isfinite(th).all()
    beta[1, 3] = float("nan")
    alpha[3, 0] = float("inf")
    S.ritz(alpha, beta, steps)
    bits = S.device_status(clear=True)
    assert bits & S.SLAQ_STATUS_NO_CONVERGENCE and bits & S.SLAQ_STATUS_NONFINITE
    t = torch.logspace(-2, 2, 40, dtype=torch.float64, device="cuda")
    S.lsd(alpha, beta, steps, 1000, t)
    assert S.device_status(clear=True) & S.SLAQ_STATUS_NO_CONVERGENCE
    S.vnge_slq(alpha, beta, steps, 1000, 900.0)
    assert S.device_status(clear=True) & S.SLAQ_STATUS_NO_CONVERGENCE
    # the closure's Gauss / Gauss-Radau rules use the same eigensolve
    th5 = torch.empty((nv, 5), dtype=torch.float64, device="cuda")
    w5 = torch.empty_like(th5)
    thr = torch.empty((nv, 6), dtype=torch.float64, device="cuda")
    wr = torch.empty_like(thr)
    S._check(S.lib().slaq_closure_rules(S._ptr(alpha), S._ptr(beta), S._ptr(steps), nv, m, 5, S._ptr(th5),
                                        S._ptr(w5), S._ptr(thr), S._ptr(wr), S._stream()))
    assert S.device_status(clear=True) & S.SLAQ_STATUS_NO_CONVERGENCE
    assert S.device_status(clear=True) == 0
