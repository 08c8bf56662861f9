"""GPU: many independent fields of uneven size and parameters in one batched call.

Batched and per-field runs execute the same kernels on the same inputs, so the
results must agree to rounding (here: exactly, the kernels are deterministic);
one 64 x 64 field of the batch is also checked against the oracle.
"""
import numpy as np
import pytest

from tests._cases import fim_err_corr, gpu_case, grad_err_sd, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import batched_fields, sample_y
    fields = batched_fields(count=6, seed=5, sides=(64, 96, 128))
    print("\n[batch]", [(w.N, w.levels) for w in fields], flush=True)
    objs = [gpu_case(w) for w in fields]
    Hs = [o[3] for o in objs]
    ys = [torch.from_numpy(sample_y(w)).cuda() for w in fields]
    thetas = np.stack([w.theta_full for w in fields])
    b = hmle.Batch(Hs)
    yield fields, objs, Hs, ys, thetas, b
    for w, m, s, H in objs:
        H.close(); s.close(); m.close()


def test_batched_equals_per_field(batch):
    fields, objs, Hs, ys, thetas, b = batch
    for ns in (1, 3):
        b.set_schedule(ns)
        ll, g, fim = b.iteration(thetas, ys)
        for f, H in enumerate(Hs):
            l1, g1, f1 = H.iteration(thetas[f], ys[f])
            # per entry, relative to each entry itself
            assert abs(ll[f] - l1) <= 1e-12 * abs(l1)
            assert np.all(np.abs(g[f] - g1) <= 1e-12 * np.abs(g1))
            assert np.all(np.abs(fim[f] - f1) <= 1e-12 * np.abs(f1))


def test_batched_field_against_oracle(batch):
    from oracle import peeling
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import Tree, dense_covariance, to_tree_order
    from synth import sample_y, sketch_draws
    fields, objs, Hs, ys, thetas, b = batch
    f = next(i for i, w in enumerate(fields) if w.N == 64)
    w = fields[f]
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, w.free)
    tree = Tree(w.dim, w.N, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, d) for d in dKs]
    om = sketch_draws(w)
    rep = peeling.build(Kt, dKt, tree, om, peeling.sketch_create(Kt, tree, om, w.rank))
    r = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, sample_y(w)))
    b.set_schedule(2)
    ll, g, fim = b.iteration(thetas, ys)
    print(f"field {f}: loglik {ll[f]!r} oracle {r['loglik']!r}")
    eg, ei = grad_err_sd(g[f], r["grad_nll"], r["fim"]), fim_err_corr(fim[f], r["fim"])
    print(f"field {f}: gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert abs(ll[f] - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eg < 1e-9
    assert ei < 1e-10


def test_batch_tune_kernels(batch):
    fields, objs, Hs, ys, thetas, b = batch
    reps = b.tune_kernels()
    shapes = {}
    for H in Hs:
        _, kc = H.sketch.ranks()
        shapes.setdefault((H.model.dim, H.model.N, H.model.leaf, kc), []).append(H.model.tuning())
    assert set(reps) == set(shapes)
    for key, choices in shapes.items():
        assert all(c == choices[0] for c in choices), key
        assert choices[0] == (reps[key]["expand_variant"], reps[key]["reduce_split_below"])
    ll, g, fim = b.iteration(thetas, ys)
    for f, H in enumerate(Hs):
        l1, g1, f1 = H.iteration(thetas[f], ys[f])
        assert rel_err(ll[f], l1) <= 1e-12


def test_batch_tune(batch):
    fields, objs, Hs, ys, thetas, b = batch
    res = b.tune(thetas, ys, candidates=(1, 2, 4))
    print(res)
    assert res["best_streams"] in (1, 2, 4)
    ll, g, fim = b.iteration(thetas, ys)
    assert np.all(np.isfinite(ll))
