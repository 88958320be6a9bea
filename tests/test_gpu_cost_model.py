"""The learned cost model: GPU gradients against the CPU reference, training,
identical counts under the learned schedule, and its gain over the
degree-product heuristic on held-out edges."""
import numpy as np
import pytest

import graphgen
import oracle
from _gpu import device, note, to_dev

pytestmark = pytest.mark.gpu


def spearman(a, b):
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))


def test_gradient_matches_cpu_reference():
    import torch

    import paper_1901_10026_amd as tg
    from oracle import mlp_ref
    dev = device()
    model = tg.CostModel(seed=5)
    rng = np.random.default_rng(5)
    params = model.get_params()
    params[tg.CostModel.num_params():tg.CostModel.num_params() + 16] = rng.normal(0, 1, 16)
    params[tg.CostModel.num_params() + 16:] = rng.uniform(0.5, 2.0, 16)
    params[:tg.CostModel.num_params()] += rng.normal(0, 0.05, tg.CostModel.num_params()).astype(np.float32)
    model.set_params(params)
    X = rng.normal(0, 2, (300, 16)).astype(np.float32)
    Y = rng.normal(3, 1, 300).astype(np.float32)
    g, loss = model.gradient(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    P = tg.CostModel.num_params()
    wq = mlp_ref.bf16_round(params[:P]).astype(np.float64)
    ref = mlp_ref.gradient(wq, params[P:], X, Y)
    ref_loss = mlp_ref.loss(wq, params[P:], X, Y)
    assert abs(float(loss.cpu()[0]) - ref_loss) <= 1e-4 * abs(ref_loss)
    # per tensor: |g - ref| <= 2^-7 |ref| + 1e-3 max|ref|
    bounds = [(0, 1024), (1024, 1088), (1088, 5184), (5184, 5248), (5248, 5312), (5312, 5313)]
    for lo, hi in bounds:
        r, q = ref[lo:hi], g[lo:hi]
        tol = 2.0 ** -7 * np.abs(r) + 1e-3 * np.abs(r).max()
        assert (np.abs(q - r) <= tol).all(), (lo, hi, np.abs(q - r).max())


@pytest.fixture(scope="module")
def trained():
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_1m()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    model = tg.CostModel(seed=55)
    note("training the cost model on a 1% edge sample")
    hist = model.train(rp, ci, ty, g.L, sample_frac=0.01, seed=56, epochs=15)
    torch.cuda.synchronize()
    return g, rp, ci, ty, model, hist


def test_training_reduces_loss(trained):
    hist = trained[5]
    note(f"loss per epoch: {[round(x, 3) for x in hist]}")
    assert hist[-1] < 0.5 * hist[0]


def test_learned_schedule_gives_identical_counts(trained):
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, model, _ = trained
    g1, r1, _ = tg.count(rp, ci, ty, g.L, schedule="degree")
    g2, r2, _ = tg.count(rp, ci, ty, g.L, schedule="learned", model=model)
    torch.cuda.synchronize()
    assert torch.equal(g1.view(torch.int64), g2.view(torch.int64))
    assert torch.equal(r1.view(torch.int64), r2.view(torch.int64))


def test_model_ranks_edge_cost_better_than_degree_product(trained):
    import torch

    import paper_1901_10026_amd as tg
    g, rp, ci, ty, model, _ = trained
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    rng = np.random.default_rng(999)          # held out: a different seed from training
    held = np.sort(rng.choice(len(ei), 20000, replace=False)).astype(np.int32)
    work = tg.edge_work(rp, ci, ty, g.L, torch.from_numpy(held).to(rp.device))
    pred = model.predict(rp, ci, ty, g.L)
    torch.cuda.synchronize()
    w = work.cpu().numpy().view(np.uint64)[held].astype(np.float64)
    pr = pred.cpu().numpy()[held]
    d = np.diff(g.row_ptr).astype(np.float64)
    heur = d[ei[held]] * d[ej[held]]
    rho_model, rho_heur = spearman(pr, w), spearman(heur, w)
    note(f"Spearman vs measured work on 20k held-out edges: model {rho_model:.3f}, d_i*d_j {rho_heur:.3f}")
    assert rho_model > rho_heur


def test_save_and_load_round_trip(trained, tmp_path):
    import paper_1901_10026_amd as tg
    model = trained[4]
    path = tmp_path / "model.bin"
    model.save(path)
    other = tg.CostModel(seed=1)
    other.load(path)
    assert np.array_equal(other.get_params(), model.get_params())


def cpu_features(g):
    """The 16 per-edge features, recomputed in numpy (float32) for every
    canonical edge: degrees, the common-neighbour type histogram and the
    combined neighbour type histogram."""
    rp, ci, ty, L = g.row_ptr.astype(np.int64), g.col_idx, g.types, g.L
    d = np.diff(rp)
    Dt = np.zeros((g.n, L), np.int64)
    for v in range(g.n):
        np.add.at(Dt[v], ty[ci[rp[v]:rp[v + 1]]], 1)
    ei, ej = oracle.canonical_edges(g.row_ptr, g.col_idx)
    F = np.zeros((len(ei), 16), np.float32)
    for e, (i, j) in enumerate(zip(ei, ej)):
        common = np.intersect1d(ci[rp[i]:rp[i + 1]], ci[rp[j]:rp[j + 1]], assume_unique=True)
        tau = np.bincount(ty[common], minlength=L).astype(np.float32)
        h8 = np.zeros(8, np.float32)
        c8 = np.zeros(8, np.float32)
        for t in range(L):
            h8[t % 8] += Dt[i, t] + Dt[j, t]
            c8[t % 8] += tau[t]
        nT = np.float32(tau.sum())
        tot = np.float32(d[i] + d[j])
        h8 = h8 / tot if tot > 0 else h8
        c8 = c8 / nT if nT > 0 else c8
        lo, hi = np.float32(min(d[i], d[j])), np.float32(max(d[i], d[j]))
        nz = h8[h8 > 0]
        F[e, 0] = np.log2(np.float32(1) + lo)
        F[e, 1] = np.log2(np.float32(1) + hi)
        F[e, 2] = np.log2(np.float32(1) + lo * hi)
        F[e, 3] = 1.0 if ty[i] == ty[j] else 0.0
        F[e, 4:12] = c8
        F[e, 12] = np.log2(np.float32(1) + nT)
        F[e, 13] = -(nz * np.log2(nz)).sum()
        F[e, 14] = h8[ty[i] % 8]
        F[e, 15] = h8[ty[j] % 8]
    return F


def test_matrix_core_inference_matches_cpu_forward():
    """Inference runs on bf16 MFMA tiles with bf16 inputs and first hidden
    layer: the CPU forward with the same roundings must agree."""
    import torch

    import paper_1901_10026_amd as tg
    from oracle import mlp_ref
    g = graphgen.chung_lu_small()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    model = tg.CostModel(seed=9)
    rng = np.random.default_rng(9)
    P = tg.CostModel.num_params()
    params = model.get_params()
    F = cpu_features(g)
    params[P:P + 16] = F.mean(axis=0)
    params[P + 16:] = np.maximum(F.std(axis=0), 1e-3)
    params[:P] += rng.normal(0, 0.1, P).astype(np.float32)
    model.set_params(params)
    pred = model.predict(rp, ci, ty, g.L)
    torch.cuda.synchronize()
    got = pred.cpu().numpy().astype(np.float64)
    w = mlp_ref.bf16_round(params[:P]).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = mlp_ref.unpack(w)
    x = mlp_ref.bf16_round(((F - params[P:P + 16]) / params[P + 16:]).astype(np.float32)).astype(np.float64)
    h1 = mlp_ref.bf16_round(np.maximum(x @ W1.T + b1, 0).astype(np.float32)).astype(np.float64)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    want = h2 @ w3 + b3
    err = np.abs(got - want)
    note(f"MFMA inference vs CPU: max abs error {err.max():.2e}, scale {np.abs(want).max():.2e}")
    assert (err <= 1e-3 + 1e-3 * np.abs(want)).all()
