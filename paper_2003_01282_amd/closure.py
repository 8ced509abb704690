"""Learned-closure pipeline on top of the C ABI (control flow only; every
numerical step runs in libslaq's kernels).

Per graph the batched engine (or the plain path, graph by graph) runs m_hi
Lanczos steps on nv probes; the first mf
coefficients of each probe give its mf-node Gauss rule (the closure's input)
and its Gauss-Radau bracket, and the full m_hi-step rule gives the training
label.  Inference needs only the mf-step run: y_hat = MLP(features), per-probe
Q_hat = Q_mf exp(y_hat) clamped to the bracket, heat = n/nv sum_p Q_hat; graphs
whose raw prediction left the bracket are flagged and recomputed by plain SLQ.
"""
import json
import os
import struct
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


def _device_pair(csr):
    return S.to_device(csr) if hasattr(csr, "row_ptr") else csr


# nonzeros per batched run (bounds the union copy of the CSR: 4 bytes each);
# every run ends on its largest graphs, so fewer, larger runs finish sooner
BATCH_NNZ = 1 << 30


# one workspace for the batched engine's global bucket per device, kept
# across plans and grown as needed (a multi-GB allocation per plan would cost
# more than the run itself on small batches)
_WS = {}


def _plan_workspace(b, device):
    nbytes = b.workspace_bytes()
    if nbytes == 0:
        return
    w = _WS.get(device)
    if w is None or w.numel() < nbytes:
        _WS.pop(device, None)
        w = S._empty_aligned(nbytes, device)
        _WS[device] = w
    b.set_workspace(w)


def _chunks(graphs):
    """Consecutive index ranges whose total nonzeros stay under BATCH_NNZ."""
    start, nnz = 0, 0
    for i, g in enumerate(graphs):
        k = int(g.nnz) if hasattr(g, "row_ptr") else int(g[1].numel())
        if i > start and nnz + k > BATCH_NNZ:
            yield start, i
            start, nnz = i, 0
        nnz += k
    if start < len(graphs):
        yield start, len(graphs)


def lanczos_batched(graphs, nv, m, seed, seeds=None):
    """alpha, beta [G nv][m] and steps [G nv] of every graph from the batched
    engine, graph i with the probes of seed + i (or seeds[i])."""
    A, B, St = [], [], []
    for lo, hi in _chunks(graphs):
        rp, ci, off = S.union_device([_device_pair(g) for g in graphs[lo:hi]])
        b = S.batch_plan_device(rp, ci, off, nv, m, 0)
        _plan_workspace(b, rp.device)
        if seeds is not None:
            b.set_seeds(torch.as_tensor(np.asarray(seeds[lo:hi], dtype=np.int64), device=rp.device))
        o = S.batch_run(b, seed + lo, heat=False, vnge=False, coeffs=True)
        A.append(o["alpha"].reshape(-1, m))
        B.append(o["beta"].reshape(-1, m))
        St.append(o["steps"].reshape(-1))
    return torch.cat(A), torch.cat(B), torch.cat(St)


def heat_batched(graphs, nv, m, t, seed, seeds=None):
    """Plain SLQ heat signatures [G][nt] of every graph from the batched
    engine (graph i with the probes of seed + i, or seeds[i])."""
    out = []
    for lo, hi in _chunks(graphs):
        rp, ci, off = S.union_device([_device_pair(g) for g in graphs[lo:hi]])
        b = S.batch_plan_device(rp, ci, off, nv, m, t.numel())
        _plan_workspace(b, rp.device)
        if seeds is not None:
            b.set_seeds(torch.as_tensor(np.asarray(seeds[lo:hi], dtype=np.int64), device=rp.device))
        out.append(S.batch_run(b, seed + lo, t, heat=True, vnge=False)["heat"])
    return torch.cat(out)


def probe_data(graphs, nv, t, m_hi=30, mf=5, seed=0, labels=True, batched=True):
    """Runs SLQ on every graph (graph i uses seed + i) and assembles the
    closure's inputs (and labels when requested).  With labels=False only mf
    steps are run (step mf also yields beta_mf, the Radau bracket's coupling).
    `graphs` holds host CSRs or (row_ptr, col_idx) device tensor pairs;
    batched=False runs the plain path graph by graph instead of the batched
    engine (same probes, same results up to summation order)."""
    m = m_hi if labels else mf
    if batched:
        alpha, beta, steps = lanczos_batched(graphs, nv, m, seed)
    else:
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
    """n/nv sum over each graph's probes (Hutchinson's estimate, in the
    library: slaq_hutchinson_mean)."""
    return S.hutchinson_mean(q.contiguous(), graph_n, nv)


def epoch_seed(seed, epoch):
    """Seed of one epoch's sample order: a function of (seed, epoch) only, so a
    run resumed at an epoch boundary draws the orders of the uninterrupted one."""
    return int(np.random.SeedSequence([int(seed), int(epoch)]).generate_state(1, dtype=np.uint64)[0] >> 1)


def train(net, data, epochs=20, batch=1024, lr=1e-3, seed=0, log=None, first_epoch=0, checkpoint=None):
    """Minibatch Adam on the kernels' train step, epochs first_epoch ..
    first_epoch + epochs - 1; with `checkpoint` (a path) the network and
    optimizer state are saved after every epoch.  Returns the loss history."""
    P = data.x.shape[0]
    gen = torch.Generator(device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for ep in range(first_epoch, first_epoch + epochs):
        gen.manual_seed(epoch_seed(seed, ep))
        perm = torch.randperm(P, device="cuda", generator=gen)
        # the epoch's loss is summed on the device and read once per epoch,
        # so the minibatch launches queue without a host wait between them
        tot = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = 0
        for s in range(0, P, batch):
            idx = perm[s:s + batch]
            net.train_step(data.x[idx].contiguous(), data.y[idx].contiguous(), lr, loss=loss)
            tot += loss
            nb += 1
        hist.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep} loss {hist[-1]:.3e}")
        if checkpoint is not None:
            save_checkpoint(net, checkpoint, epoch=ep + 1, seed=seed)
    return hist


CHECKPOINT_FORMAT = "slaq-closure-checkpoint-1"
_CKPT_ARRAYS = (("weights", 0), ("adam_m1", 2), ("adam_m2", 3))


def save_checkpoint(net, path, epoch=0, seed=0):
    """Network and optimizer state as one file: an 8-byte little-endian
    header length, a JSON header (shape, Adam step count, epochs completed,
    shuffling seed, array names), then the FP32 weights and the two Adam
    moment vectors, little-endian, n_params values each."""
    header = {"format": CHECKPOINT_FORMAT, "d_in": net.d_in, "hidden": net.hidden, "nt": net.nt,
              "n_params": net.n_params, "offsets": net.offsets, "dims": net.dims, "adam_step": net.step(),
              "epoch": int(epoch), "seed": int(seed), "arrays": [a for a, _ in _CKPT_ARRAYS], "dtype": "<f4"}
    head = json.dumps(header).encode()
    tmp = f"{path}.tmp"
    with open(tmp, "wb") as f:
        f.write(struct.pack("<Q", len(head)))
        f.write(head)
        for _, which in _CKPT_ARRAYS:
            f.write(net.get(which).cpu().numpy().astype("<f4").tobytes())
    os.replace(tmp, path)


def load_checkpoint(path):
    """A new network with the checkpoint's weights and optimizer state, and
    the header (its "epoch" is the first_epoch to resume training at)."""
    with open(path, "rb") as f:
        (hl,) = struct.unpack("<Q", f.read(8))
        header = json.loads(f.read(hl).decode())
        if header.get("format") != CHECKPOINT_FORMAT:
            raise ValueError(f"{path}: not a closure checkpoint ({header.get('format')!r})")
        P = int(header["n_params"])
        vecs = {}
        for name in header["arrays"]:
            buf = f.read(4 * P)
            if len(buf) != 4 * P:
                raise ValueError(f"{path}: truncated at {name}")
            vecs[name] = np.frombuffer(buf, dtype="<f4").astype(np.float32)
        if f.read(1):
            raise ValueError(f"{path}: trailing bytes")
    # the file is whole: only now is the device touched
    vecs = {k: torch.from_numpy(v).cuda() for k, v in vecs.items()}
    net = S.Closure(d_in=header["d_in"], hidden=header["hidden"], nt=header["nt"])
    if net.n_params != P or net.offsets != header["offsets"] or net.dims != header["dims"]:
        raise ValueError(f"{path}: parameter layout does not match this library")
    net.set(vecs["weights"], reset_optimizer=False)
    net.set_optimizer(vecs["adam_m1"], vecs["adam_m2"], header["adam_step"])
    return net, header


def infer(net, data, tol=1e-3):
    """Closure heat per graph and the graphs flagged for plain SLQ."""
    yhat = net.forward(data.x)
    return S.closure_apply(yhat, data.q5, data.qr, data.graph_n, data.nv, tol)


def heat_with_fallback(net, data, graphs, nv, t, seed=0, tol=1e-3, m_plain=30, batched=True):
    """Closure heat, with every flagged graph recomputed by plain SLQ
    (m_plain steps, same probes: graph i uses seed + i), in one batched run
    (or graph by graph with batched=False).  Returns host arrays."""
    heat, flags = infer(net, data, tol)
    heat = heat.cpu().numpy()
    flags = flags.cpu().numpy()
    idx = np.flatnonzero(flags)
    if idx.size and batched:
        sel = [graphs[i] for i in idx]
        heat[idx] = heat_batched(sel, nv, m_plain, t, 0, seeds=seed + idx).cpu().numpy()
    else:
        for i in idx:
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
