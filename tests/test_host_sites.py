"""Host logic of the SN hand-over (Sec. 3.2): the site selection keeps, in
draw order, every candidate whose box overlaps no box kept before it.  The
selection sorts each draw by x and tests only the kept sites inside an x
window; here it is held to the plain rule (test against every kept site)
on synthetic draws, sparse and crowded, over several draws."""
import numpy as np
import pytest

from paper_2510_23330_amd.coupling import keep_in_order


def _plain(draws, P, side, want):
    kept, chosen, seen = [], [], set()
    for draw in draws:
        for d in draw.tolist():
            if d in seen:
                continue
            seen.add(d)
            p = P[d]
            if any(np.all(np.abs(p - q) < side) for q in kept):
                continue
            kept.append(p)
            chosen.append(d)
            if len(chosen) == want:
                return chosen
    return chosen


def _fast(draws, P, side, want):
    kept, chosen, seen = np.zeros((0, 3)), [], set()
    for draw in draws:
        kept = keep_in_order(draw, P[draw], side, kept, seen, chosen, want)
        assert kept.shape == (len(chosen), 3)
        if len(chosen) == want:
            break
    return chosen


@pytest.mark.parametrize("scale", [15.0, 0.3, 0.06, 0.01])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_site_selection_matches_plain_rule(scale, seed):
    rng = np.random.default_rng(seed)
    n, K, side = 20000, 64, 0.06
    R = scale * np.sqrt(rng.random(n))
    ph = 2 * np.pi * rng.random(n)
    P = np.stack([R * np.cos(ph), R * np.sin(ph), 0.01 * scale * (rng.random(n) - 0.5)], 1)
    # some exact coincidences and points exactly `side` apart on x
    P[1] = P[0]
    P[3] = P[2] + np.array([side, 0.0, 0.0])
    draws = [np.concatenate([[0, 1, 2, 3], rng.choice(np.arange(4, n), 4 * K - 4, replace=False)])]
    draws += [rng.choice(n, 4 * K, replace=False) for _ in range(6)]
    a = _plain(draws, P, side, K)
    b = _fast(draws, P, side, K)
    assert a == b
    assert len(set(b)) == len(b)
    Q = P[b]
    for i in range(len(b)):  # no two kept boxes overlap
        d = np.abs(Q - Q[i]) < side
        assert np.count_nonzero(d.all(axis=1)) == 1
