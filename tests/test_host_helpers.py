"""Host-side logic checked on the CPU: the H-matvec used by the full-size GPU checks
agrees with the dense matrix of the same representation, and the batched workload's
longest-first placement of fields on streams (hmle.place_fields) is a balanced,
complete assignment."""
import numpy as np

from tests._cases import densify, hmatvec


def test_hmatvec_matches_densify():
    rng = np.random.default_rng(0)
    levels, kc, n = 3, 5, 64
    F = rng.standard_normal((levels * kc, n))
    dF = rng.standard_normal((levels * kc, n))
    nl = n >> levels
    lv = rng.standard_normal((1 << levels, nl, nl))
    dlv = rng.standard_normal((1 << levels, nl, nl))
    x = rng.standard_normal((n, 3))
    K = densify(F, lv, levels, kc, n)
    dK = densify(F, dlv, levels, kc, n, dF=dF)
    assert np.abs(hmatvec(F, lv, levels, kc, x) - K @ x).max() < 1e-12 * np.abs(K).max() * n
    assert np.abs(hmatvec(F, lv, levels, kc, x[:, 1]) - K @ x[:, 1]).max() < 1e-12 * np.abs(K).max() * n
    got = hmatvec(F, lv, levels, kc, x, dF=dF, dleaves=dlv)
    assert np.abs(got - dK @ x).max() < 1e-12 * np.abs(dK).max() * n


def test_densify_block_layout():
    # one level, kc = 1: the off-diagonal block is the outer product of the two halves
    n = 4
    F = np.array([[1.0, 2.0, 3.0, 4.0]])
    lv = np.zeros((2, 2, 2))
    K = densify(F, lv, 1, 1, n)
    assert np.array_equal(K[:2, 2:], np.outer([1.0, 2.0], [3.0, 4.0]))
    assert np.array_equal(K[2:, :2], np.outer([3.0, 4.0], [1.0, 2.0]))


def test_place_fields_longest_first():
    from paper_2303_10102_amd.hmle import place_fields
    rng = np.random.default_rng(3)
    cost = list(rng.uniform(1.0, 100.0, size=23))
    for ns in (1, 2, 4, 8):
        lanes, order = place_fields(cost, ns)
        assert len(lanes) == ns
        assert sorted(order) == list(range(len(cost)))            # every field once
        assert sorted(f for lane in lanes for f in lane) == list(range(len(cost)))
        loads = [sum(cost[f] for f in lane) for lane in lanes]
        # longest-processing-time bound: no stream exceeds the mean load by more than the
        # largest single cost
        assert max(loads) <= sum(cost) / ns + max(cost) + 1e-9
        for lane in lanes:                                        # each lane longest first
            assert all(cost[a] >= cost[b] for a, b in zip(lane, lane[1:]))
        # the enqueue order starts every stream before any stream's second field
        firsts = {lane[0] for lane in lanes if lane}
        assert set(order[:len(firsts)]) == firsts
    # more streams than fields: the extra streams stay empty
    lanes, order = place_fields([5.0, 1.0], 4)
    assert lanes == [[0], [1], [], []] and order == [0, 1]
