"""Learned-closure pipeline on top of the C ABI (control flow only; every
numerical step runs in libslaq's kernels).

Per graph the plain path runs m_hi Lanczos steps on nv probes; the first mf
coefficients of each probe give its mf-node Gauss rule (the closure's input)
and its Gauss-Radau bracket, and the full m_hi-step rule gives the training
label.  Inference needs only the mf-step run: y_hat = MLP(features), per-probe
Q_hat = Q_mf exp(y_hat) clamped to the bracket, heat = n/nv sum_p Q_hat; graphs
whose raw prediction left the bracket are flagged and recomputed by plain SLQ.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import slaq as S


@dataclass
class ProbeData:
    x: torch.Tensor        # BF16 features [P][32]
    q5: torch.Tensor       # Gauss values of the mf-node rule [P][nt]
    qr: torch.Tensor       # Gauss-Radau upper values [P][nt]
    q_hi: torch.Tensor     # Gauss values of the m_hi-node rule [P][nt] (labels); None for inference
    y: torch.Tensor        # targets log q_hi - log q5 [P][nt]; None for inference
    graph_n: torch.Tensor  # node counts [G] (int64, device)
    nv: int


def graph_nodes(csr):
    return csr.n if hasattr(csr, "n") else csr[0].numel() - 1


def lanczos_graph(csr, nv, m, seed):
    rp, ci = S.to_device(csr) if hasattr(csr, "row_ptr") else csr
    g = S.build_graph(rp, ci)
    return S.lanczos(g, nv, m, seed)


def probe_data(graphs, nv, t, m_hi=30, mf=5, seed=0, labels=True):
    """Runs the plain path per graph (graph i uses seed + i) and assembles the
    closure's inputs (and labels when requested).  With labels=False only mf
    steps are run (step mf also yields beta_mf, the Radau bracket's coupling).
    `graphs` holds host CSRs or (row_ptr, col_idx) device tensor pairs."""
    m = m_hi if labels else mf
    A, B, St = [], [], []
    for i, csr in enumerate(graphs):
        a, b, s = lanczos_graph(csr, nv, m, seed + i)
        A.append(a)
        B.append(b)
        St.append(s)
    alpha = torch.cat(A)
    beta = torch.cat(B)
    steps = torch.cat(St)
    th5, w5, thr, wr = S.closure_rules(alpha, beta, steps, mf=mf)
    x = S.closure_features(th5, w5)
    q5 = S.gauss_values(th5, w5, t)
    qr = S.gauss_values(thr, wr, t)
    q_hi = y = None
    if labels:
        th, w2 = S.ritz(alpha, beta, steps)
        q_hi = S.gauss_values(th, w2, t)
        y = S.closure_targets(q_hi, q5)
    gn = torch.tensor([graph_nodes(c) for c in graphs], dtype=torch.int64, device="cuda")
    return ProbeData(x=x, q5=q5, qr=qr, q_hi=q_hi, y=y, graph_n=gn, nv=nv)


def heat_from_q(q, graph_n, nv):
    """n/nv sum over each graph's probes (plain Hutchinson aggregation)."""
    G = graph_n.numel()
    return q.view(G, nv, -1).sum(dim=1) * (graph_n.to(torch.float64) / nv)[:, None]


def train(net, data, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Minibatch Adam on the kernels' train step; returns the loss history."""
    P = data.x.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(P, device="cuda", generator=gen)
        tot, nb = 0.0, 0
        for s in range(0, P, batch):
            idx = perm[s:s + batch]
            net.train_step(data.x[idx].contiguous(), data.y[idx].contiguous(), lr, loss=loss)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep} loss {hist[-1]:.3e}")
    return hist


def infer(net, data, tol=1e-3):
    """Closure heat per graph and the graphs flagged for plain SLQ."""
    yhat = net.forward(data.x)
    return S.closure_apply(yhat, data.q5, data.qr, data.graph_n, data.nv, tol)


def heat_with_fallback(net, data, graphs, nv, t, seed=0, tol=1e-3, m_plain=30):
    """Closure heat, with every flagged graph recomputed by plain SLQ
    (m_plain steps, same probes: graph i uses seed + i).  Returns host arrays."""
    heat, flags = infer(net, data, tol)
    heat = heat.cpu().numpy()
    flags = flags.cpu().numpy()
    for i in np.flatnonzero(flags):
        a, b, s = lanczos_graph(graphs[i], nv, m_plain, seed + i)
        th, w2 = S.ritz(a, b, s)
        heat[i] = S.signature(th, w2, graph_nodes(graphs[i]), t).cpu().numpy()
    return heat, flags


def tune_gate(net, dval, nv, candidates=(1e-3, 2e-3, 5e-3, 1e-2, 2e-2, 5e-2, 1e-1, 1.0),
              target=1e-3, min_ok=0.99):
    """Largest gate tolerance whose outcome on validation graphs keeps at
    least `min_ok` of them within `target` (relative l2 against the labels,
    plain m_hi SLQ on the same probes; flagged graphs count as exact since
    they fall back to it).  Returns (tolerance, table)."""
    ref = heat_from_q(dval.q_hi, dval.graph_n, nv).cpu().numpy()
    table = []
    best = None
    for tol in sorted(candidates):
        heat, flags = infer(net, dval, tol)
        e = rel_l2(heat.cpu().numpy(), ref)
        f = flags.cpu().numpy().astype(bool)
        ok = float(np.mean(np.where(f, True, e <= target)))
        table.append({"tol": tol, "fallback": float(f.mean()), "ok": ok})
        if ok >= min_ok:
            best = tol
    return (best if best is not None else min(candidates)), table


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)
