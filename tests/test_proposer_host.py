"""Training targets of the learned proposer, on the host (CPU).

``proposer.cell_labels`` labels each training injection with the cell of its (Mc, q) in the
neighbourhood of the coarse template that found it.  The model is trained on these labels and
its selection is applied through the cell rule of the follow-up, so the labels must be that rule:
checked against the oracle's ``cell_index`` on random points and on exact bin and q edges, and,
outside the neighbourhood (where the rule has no cell), clamped to the nearest edge bin.
"""
import numpy as np

from oracle import proposer as P

Q_EDGES = (1.75, 2.5, 3.25)
FRAC = 0.05


def test_cell_labels_equal_the_oracle_cell_rule():
    from paper_2309_00019_amd import proposer
    g = np.random.default_rng(7)
    mc_c = g.uniform(1.2, 10.0, 4000)
    mc_f = mc_c * (1.0 + FRAC * g.uniform(-1.0, 1.0, 4000))
    q_f = g.uniform(1.0, 4.0, 4000)
    # exact edges: u = -1, -7/8, 0, 1/8, 1 and q on each edge
    for u in (-1.0, -0.875, 0.0, 0.125, 1.0):
        for q in Q_EDGES + (1.0, 4.0):
            mc_c = np.append(mc_c, 2.0)
            mc_f = np.append(mc_f, 2.0 + u * FRAC * 2.0)
            q_f = np.append(q_f, q)
    got = proposer.cell_labels(mc_c, mc_f, q_f, FRAC, Q_EDGES)
    ref = np.array([P.cell_index(a, b, c, FRAC, Q_EDGES) for a, b, c in zip(mc_c, mc_f, q_f)])
    inside = ref >= 0
    # only the points built on the neighbourhood's ends (u = +-1, not exact in binary) may fall
    # outside by rounding; there the label is the clamped end bin
    assert inside[:4000].all() and inside.sum() >= len(ref) - 10
    assert np.array_equal(got[inside], ref[inside])
    assert np.all(np.isin(got[~inside] // 4, (0, 15)))
    assert set(np.unique(got[inside])) == set(range(64))   # every cell is reached


def test_cell_labels_clamp_outside_the_neighbourhood():
    from paper_2309_00019_amd import proposer
    mc_c = np.array([3.0, 3.0])
    mc_f = np.array([3.0 * (1 - 3 * FRAC), 3.0 * (1 + 3 * FRAC)])
    q_f = np.array([1.2, 3.9])
    assert [P.cell_index(a, b, c, FRAC, Q_EDGES) for a, b, c in zip(mc_c, mc_f, q_f)] == [-1, -1]
    assert proposer.cell_labels(mc_c, mc_f, q_f, FRAC, Q_EDGES).tolist() == [4 * 0 + 0, 4 * 15 + 3]
