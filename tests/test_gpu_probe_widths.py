"""Every probe-block width against the oracle: nv from 1 to 70 gives lane
groups of 1 to 64 lanes (wave split into 64 // groups of them, with lanes left
over when the width does not divide 64), one or two probe tiles, and
the padding of the last quad; each width's alpha, beta and step counts
against the FP64 oracle on the same probes (§3.1's recurrence), with
relabelling (heavy rows cut into pieces) and without."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 3, 5, 7, 9, 11, 13, 17, 20, 23, 28, 33, 41, 50, 64, 65, 70]


@pytest.fixture(scope="module")
def graph():
    csr = inputs.rmat(13, seed=21)
    return csr, O.build_graph(csr.n, csr.row_ptr, csr.col_idx)


@pytest.mark.parametrize("relabel", [True, False])
def test_every_probe_width_against_oracle(graph, relabel):
    csr, og = graph
    m, seed = 5, 404
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci, relabel=relabel)
    g.set_fused(0)
    print(f"\n[gpu] probe widths relabel={relabel}: n={csr.n} nnz={csr.nnz}", flush=True)
    for nv in WIDTHS:
        a, b, st = S.lanczos(g, nv, m, seed)
        torch.cuda.synchronize()
        assert S.device_status(clear=True) == 0, nv
        oa, ob, os_ = O.lanczos(og, nv, m, seed)
        np.testing.assert_array_equal(st.cpu().numpy(), os_, err_msg=f"nv={nv}")
        np.testing.assert_allclose(a.cpu().numpy(), oa, rtol=1e-5, atol=1e-6, err_msg=f"alpha nv={nv}")
        np.testing.assert_allclose(b.cpu().numpy(), ob, rtol=1e-5, atol=1e-6, err_msg=f"beta nv={nv}")
