"""Parity of what the benchmark times: every workload at its full size, run through
its instance (same inputs, same calls) with the variants the tuning table selects,
checked against the FP64 oracle -- in full where the oracle is cheap, otherwise on
sampled rows (products) or sampled column sets (correlation, covariance, SYRK),
whose outputs depend on the sampled rows/columns only.

Covered: every batch instance at all five sizes with the table's variants; every
non-default feature-reuse assignment (K = 1 and 3) on the instances it serves; the
replayed graph of the tuned batch at 256, 512 and 1000 (each instance against the
oracle after the first replay, and bitwise equal after the second); the precision
workloads and the next rows."""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_1810_10496_amd import api, synth, tuned, workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"fp32": 1e-4, "bf16": 2e-2, "split": 1e-5}


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    c = api.context(0)
    applied = tuned.apply(c)
    assert all(e["vid"] >= 0 for e in applied), "a table entry could not be loaded"
    return c


def _sample(n, k, seed):
    s = np.unique(synth.splitmix64(seed, 0, k) % np.uint64(n)).astype(np.int64)
    return np.unique(np.concatenate([s, [0, n - 1]]))


def _instances():
    out = W.batch_instances(W.SIZES) + W.config_instances() + W.precision_instances((4096,)) + \
        W.corr_precision_instances((4096,)) + W.next_instances()
    seen, uniq = set(), []
    for i in out:
        if i.name not in seen:
            seen.add(i.name)
            uniq.append(i)
    return uniq


INSTANCES = _instances()


def _prec(name):
    return "bf16" if "bf16" in name else ("split" if "split" in name else "fp32")


def _run(ctx, inst):
    st = inst.make(DEV, 1)
    before = {k: (v[0].clone() if isinstance(v, list) else v.clone())
              for k, v in st.items() if isinstance(v, (list, torch.Tensor)) and k != "ws"}
    stream = torch.cuda.current_stream()
    inst.run(ctx, st, 0, stream)
    torch.cuda.synchronize()
    return st, {k: h(v) for k, v in before.items()}


def check(inst, st, x):
    """(error, tolerance) of the instance's outputs in `st` against the oracle on the
    inputs `x` (host copies taken before the run)."""
    op, n, prec = inst.op, inst.size, _prec(inst.name)
    tol = TOL[prec]
    if op.startswith("gemm3"):
        rows = _sample(n, 16, 7001)
        A, B, C, D = x["A"], x["B"], x["C"], x["D"]
        a, b = st["alpha"], st["beta"]
        ref = o.gemm3(A[rows], B, C, D[rows], a, b)
        err = o.max_err(h(st["D"][0])[rows], ref, o.gemm3_scale(A[rows], B, C, D[rows], a, b))
    elif op.startswith("gemm"):
        rows = _sample(n, 24, 7002)
        A, B, C = x["A"], x["B"], x["C"]
        a, b = st["alpha"], st["beta"]
        ref = o.gemm(A[rows], B, C[rows], a, b)
        err = o.max_err(h(st["C"][0])[rows], ref, o.gemm_scale(A[rows], B, C[rows], a, b))
    elif op in ("gemv", "gemv_t", "gemv_pair"):
        A = x["A"]
        errs = []
        if op in ("gemv", "gemv_pair"):
            errs.append(o.max_err(h(st["y1"]), o.gemv(A, x["x"])))
        if op in ("gemv_t", "gemv_pair"):
            errs.append(o.max_err(h(st["y2"]), o.gemv_t(A, x["z"])))
        err = max(errs)
    elif op in ("conv2d", "conv3d"):
        grid, taps = x["inp"], st["taps"]
        f = o.conv2d if op == "conv2d" else o.conv3d
        err = o.max_err(h(st["out"][0]), f(grid, taps), f(np.abs(grid), np.abs(taps)))
    elif op == "colstats":
        mu, sd = o.colstats(x["X"], st["eps"])
        assert o.max_err(h(st["mu"]), mu, o.colstats(np.abs(x["X"]), st["eps"])[0]) <= 1e-6
        err = o.max_err(h(st["sd"]), sd)
        tol = 1e-5
    elif op.startswith("corr"):
        cols = _sample(n, 24, 7003)
        Rs, S = o.corr(x["X"][:, cols], st["eps"], with_scale=True)
        R = h(st["R"])
        assert np.array_equal(R, R.T)
        err = o.max_err(R[np.ix_(cols, cols)], Rs, S)
    elif op == "covar":
        cols = _sample(n, 24, 7004)
        Xs = x["X"][:, cols]
        Xc = Xs.astype(np.float64) - Xs.astype(np.float64).mean(axis=0)
        scale = np.abs(Xc).T @ np.abs(Xc) / (n - 1)
        Cg = h(st["C"])
        assert np.array_equal(Cg, Cg.T)
        err = o.max_err(Cg[np.ix_(cols, cols)], o.covar(Xs), scale)
    elif op in ("syrk", "syr2k"):
        rows = _sample(n, 24, 7005)
        ix = np.ix_(rows, rows)
        A, C0 = x["A"][rows], x["C"][ix]
        if op == "syrk":
            ref, s = o.syrk(A, C0, 1.5, 1.2), o.syrk(np.abs(A), np.abs(C0), 1.5, 1.2)
        else:
            B = x["B"][rows]
            ref, s = o.syr2k(A, B, C0, 1.5, 1.2), o.syr2k(np.abs(A), np.abs(B), np.abs(C0), 1.5, 1.2)
        err = o.max_err(h(st["C"][0])[ix], ref, s)
    elif op == "gesummv":
        A, B, xv = x["A"], x["B"], x["x"]
        err = o.max_err(h(st["y"]), o.gesummv(A, B, xv, 1.5, 1.2),
                        o.gesummv(np.abs(A), np.abs(B), np.abs(xv), 1.5, 1.2))
    elif op == "mvt":
        A = x["A"]
        r1, r2 = o.mvt(A, x["y1"], x["y2"], x["x1"], x["x2"])
        s1, s2 = o.mvt(np.abs(A), np.abs(x["y1"]), np.abs(x["y2"]), np.abs(x["x1"]), np.abs(x["x2"]))
        err = max(o.max_err(h(st["x1"]), r1, s1), o.max_err(h(st["x2"]), r2, s2))
    elif op == "fdtd2d":
        T = x["fict"].shape[0]
        refs, scales = o.fdtd2d(x["fict"], x["ex"], x["ey"], x["hz"], with_scale=True)
        err = max(o.max_err(h(st[key][0]), ref, sc) for key, ref, sc in zip(("ex", "ey", "hz"), refs, scales))
        tol = 1e-6 * (1 + T)    # per element, against the term magnitudes of its domain of dependence
    else:
        raise AssertionError(f"no check for {inst.name}")
    return err, tol


@pytest.mark.parametrize("inst", INSTANCES, ids=[i.name for i in INSTANCES])
def test_tuned_workload_vs_oracle(ctx, inst):
    print("[case] tuned", inst.name, flush=True)
    st, x = _run(ctx, inst)
    err, tol = check(inst, st, x)
    print("[case] tuned", inst.name, "err", err, flush=True)
    assert err <= tol


# ------------------------------------------------------------------ feature reuse --

def _reuse_cases():
    """(instance, K) for every batch instance one of whose families has a non-default
    reuse assignment at its size."""
    nondef = {(e["family"], int(e["size"]), int(e["k"])) for e in tuned.read_reuse() if not e.get("is_default")}
    out = []
    for inst in W.batch_instances(W.SIZES):
        for k in (1, 3):
            if any((f, inst.size, k) in nondef for f in inst.families):
                out.append((inst, k))
    return out


REUSE = _reuse_cases()


@pytest.fixture(scope="module")
def reuse(ctx):
    return tuned.load_reuse(ctx)


def test_every_reuse_assignment_is_exercised():
    """Each non-default assignment is reachable through an instance of the batch."""
    want = {(e["family"], int(e["size"]), int(e["k"])) for e in tuned.read_reuse() if not e.get("is_default")}
    got = {(f, inst.size, k) for inst, k in REUSE for f in inst.families}
    assert want <= got


@pytest.mark.parametrize("inst,k", REUSE, ids=[f"{i.name}-k{k}" for i, k in REUSE])
def test_reuse_variant_vs_oracle(ctx, reuse, inst, k):
    print("[case] reuse", inst.name, "K", k, flush=True)
    vids = {f: reuse.get((f, inst.size, k)) for f in inst.families}
    assert all(v is not None for v in vids.values()), "a reuse code object could not be loaded"
    for f, v in vids.items():
        ctx.variant_select(f, v)
    try:
        st, x = _run(ctx, inst)
    finally:
        for f in vids:
            ctx.variant_select(f, -1)
    err, tol = check(inst, st, x)
    print("[case] reuse", inst.name, "K", k, "err", err, flush=True)
    assert err <= tol


# --------------------------------------------------------- the replayed tuned batch --

def test_tuned_batch_graph_vs_oracle(ctx):
    """The batch at 256, 512 and 1000 captured into one graph with the table's variants
    (as the benchmark captures it), replayed: every instance against the oracle after the
    first replay; after restoring the in-place operands and doing eager work, a second
    replay gives the same bits."""
    insts = W.batch_instances((256, 512, 1000))
    stream = torch.cuda.Stream()
    states, before = [], []
    for inst in insts:
        st = inst.make(DEV, 1)
        states.append(st)
        before.append({k: (v[0].clone() if isinstance(v, list) else v.clone())
                       for k, v in st.items() if isinstance(v, (list, torch.Tensor)) and k != "ws"})
    torch.cuda.synchronize()
    with ctx.capture(stream) as graph:
        for inst, st in zip(insts, states):
            inst.run(ctx, st, 0, stream)
    print(f"[case] tuned batch graph of {len(insts)} instances captured", flush=True)

    def outputs(st):
        return {k: h(v[0] if isinstance(v, list) else v) for k, v in st.items()
                if isinstance(v, (list, torch.Tensor)) and k != "ws"}

    graph.launch(stream)
    stream.synchronize()
    first = []
    for inst, st, b in zip(insts, states, before):
        x = {k: h(v) for k, v in b.items()}
        err, tol = check(inst, st, x)
        print("[case] graph", inst.name, "err", err, flush=True)
        assert err <= tol, inst.name
        first.append(outputs(st))
    for st, b in zip(states, before):         # in-place operands (C, D) back to their inputs
        for k, v in b.items():
            (st[k][0] if isinstance(st[k], list) else st[k]).copy_(v)
    torch.ones(1 << 20, device=DEV).mul_(2.0)  # eager work between the replays
    torch.cuda.synchronize()
    graph.launch(stream)
    stream.synchronize()
    for inst, st, f in zip(insts, states, first):
        for k, v in outputs(st).items():
            assert np.array_equal(v, f[k]), (inst.name, k)
    graph.destroy()


# ------------------------------------------------------------------ phase orders --

ORDERS = tuned.read_orders()


def test_every_phase_order_entry_builds():
    """Each minimal best order of the phase-order exploration reproduces its recorded
    code object (the benchmark times exactly that code)."""
    for e in ORDERS:
        assert tuned.code_for(e) is not None, e["family"]


@pytest.mark.parametrize("e", ORDERS, ids=[e["family"] for e in ORDERS])
def test_phase_order_vs_oracle(ctx, e):
    """The family's best phase order (default knobs) on the instance the benchmark times
    it on, against the oracle."""
    fam = e["family"]
    vid = ctx.variant_load(tuned.code_for(e))
    try:
        for inst in W.family_instances(fam, (e["size"],)):
            print("[case] phase order", fam, inst.name, flush=True)
            ctx.variant_select(fam, vid)
            try:
                st, x = _run(ctx, inst)
            finally:
                ctx.variant_select(fam, -1)
            err, tol = check(inst, st, x)
            print("[case] phase order", fam, inst.name, "err", err, flush=True)
            assert err <= tol
    finally:
        ctx.variant_unload(vid)
