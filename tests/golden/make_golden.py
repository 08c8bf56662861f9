"""Write the stored oracle values of the small parity cases (tests/golden/*.json).

Every number comes from oracle/ applied to the seeded synth/ inputs; nothing here
touches the HIP library.  What is stored, per case:
  * the HODLR approximation's log-likelihood, log-determinant, negative score and
    expected Fisher matrix (Sec. 4.1 eq. "log-like approximated", Sec. 4.3 eqs.
    "score approximated" and "fisher info approximated"), with K~ and its derivative
    matrices built by the peeling replay of Alg. 1 and Alg. 2;
  * the same quantities for the exact covariance K (Sec. 2 eqs. "log-like", "score",
    "fisher info"), as the reference of the approximation.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import peeling  # noqa: E402
from oracle.exact import likelihood_gradient_fisher  # noqa: E402
from oracle.model import Tree, dense_covariance, to_tree_order  # noqa: E402
from synth import sample_y, sketch_draws  # noqa: E402

KEYS = ("1d_n1024", "2d_n1024")


def case_values(w):
    y = sample_y(w)
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, w.free)
    tree = Tree(w.dim, w.N, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, d) for d in dKs]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    rep = peeling.build(Kt, dKt, tree, om, V)
    yt = to_tree_order(tree, y)
    approx = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], yt)
    exact = likelihood_gradient_fisher(Kt, dKt, yt)

    def pick(r):
        return {"loglik": r["loglik"], "logdet": r["logdet"], "grad_nll": [float(v) for v in r["grad_nll"]],
                "fim": [[float(v) for v in row] for row in r["fim"]]}

    return {"case": w.name, "n": int(w.n), "params": list(w.free), "theta": [float(t) for t in w.theta_full],
            "hodlr": pick(approx), "exact": pick(exact)}


def main():
    from tests._cases import CASES
    for key in KEYS:
        vals = case_values(CASES[key])
        vals["source"] = ("oracle/ (peeling replay of Alg. 1 and Alg. 2; dense L, score and expected "
                          "Fisher from their definitions) on synth/ inputs; tests/golden/make_golden.py")
        with open(os.path.join(HERE, f"oracle_{key}.json"), "w") as fh:
            json.dump(vals, fh, indent=1)
            fh.write("\n")
        print("wrote", key, vals["hodlr"]["loglik"])


if __name__ == "__main__":
    main()
