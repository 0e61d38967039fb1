"""Forced near-ties for the tests of the near-tie protocol.

A trial is a near-tie when its uniform u lies within 1e-12 of its
acceptance probability exp(-beta dE) (Supplementary, "Monte Carlo Simulation
Algorithms", the acceptance rule; the 1e-12 window is this library's
convention).  Random inputs never come that close, so these helpers build
one: they take a trial of mini-step 0 (whose energy change depends only on
the initial configuration, since the trials of a mini-step are
independent), draw its Philox block, and choose beta = -log(u) / dE, which
puts exp(-beta dE) within a few ulps of u.  Everything comes from the oracle
(Philox, partner, dE) and the seeded inputs; nothing from the HIP path.
"""
import math

import numpy as np

from oracle import oracle as O

TIE_WINDOW = 1e-12


def u53(w) -> float:
    """The 53-bit uniform (w1 2^21 + floor(w2 / 2^11)) 2^-53 of a Philox block."""
    return float((int(w[1]) << 21) | (int(w[2]) >> 11)) * 2.0 ** -53


def trial_draw(seed: int, replica: int, sweep: int, site: int, Z1: int):
    """Philox4x32-10 of the trial at `site` (counter (site, sweep, replica),
    key seed): the partner direction k and the uniform u."""
    w = O.philox([site & 0xFFFFFFFF, site >> 32, sweep, replica & 0xFFFFFFFF],
                 [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return (int(w[0]) * Z1) >> 32, u53(w)


def exchange_draw(seed: int, round_: int, pair: int) -> float:
    """The uniform of slot pair `pair` in exchange round `round_` (counter
    (pair, 0, round, 0xffffffff))."""
    w = O.philox([pair, 0, round_, 0xFFFFFFFF], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return u53(w)


def ministep0_sites(lattice: int, dims, cells):
    """Active sites of mini-step 0 (basis site 0 at every link-cell origin),
    cells x fastest, then y, then z."""
    m = 2 if lattice == 0 else 4
    org = [np.concatenate([[0], np.cumsum(np.asarray(c, np.int64))[:-1]]) for c in cells]
    for z in org[2]:
        for y in org[1]:
            for x in org[0]:
                yield int(m * (x + dims[0] * (y + dims[1] * z)))


def forced_trial_tie(lattice: int, dims, K: int, S: int, cells, occ, V, seed: int, replica: int = 0,
                     sweep: int = 0, W=None, skip: int = 0, u_lo: float = 0.05, u_hi: float = 0.95):
    """A trial of mini-step 0 of (replica, sweep) with dE > 0 and u in
    (u_lo, u_hi), and the inverse temperature that makes it a near-tie.

    Returns dict(site, k, partner, dE, u, beta, P) with P = exp(-beta dE)
    formed as the sweep forms it (x = beta * dE in binary64, then exp(-x)).
    `skip` passes over that many candidates first.  W selects the qSRO
    energy change instead of the pair model's."""
    Z1 = int(O.shells(lattice, 1)[0][0])
    for a in ministep0_sites(lattice, dims, cells):
        k, u = trial_draw(seed, replica, sweep, a, Z1)
        if not (u_lo < u < u_hi):
            continue
        if W is None:
            dE, b = O.delta_e(lattice, dims, K, S, occ, V, a, k)
        else:
            dE, b = O.qsro_delta_e(lattice, dims, K, S, occ, V, W, a, k)
        if not dE > 0.0:
            continue
        beta = -math.log(u) / dE
        P = math.exp(-(beta * dE))
        if abs(u - P) >= 1e-3 * TIE_WINDOW:
            continue
        if skip > 0:
            skip -= 1
            continue
        return dict(site=a, k=k, partner=b, dE=dE, u=u, beta=beta, P=P)
    raise AssertionError("no candidate trial for a forced near-tie")


def forced_exchange_tie(E, beta_slot, rep_at, seed: int, round_: int, pair: int):
    """Inverse temperatures of the slots with pair (pair, pair + 1) of round
    `round_` at a near-tie: beta_slot[pair + 1] is moved so that
    x = (beta_slot[pair] - beta_slot[pair + 1]) (E[a] - E[b]) has
    |u - exp(x)| < 1e-12 and x < 0.  Returns (new beta_slot, u, x)."""
    bs = np.array(beta_slot, np.float64)
    a, b = int(rep_at[pair]), int(rep_at[pair + 1])
    dEab = float(E[a]) - float(E[b])
    assert dEab != 0.0
    u = exchange_draw(seed, round_, pair)
    bs[pair + 1] = bs[pair] - math.log(u) / dEab
    x = (bs[pair] - bs[pair + 1]) * dEab
    # x carries the rounding of the beta difference (a few 1e-14 relative);
    # well inside the window, where either side's exp rounding cannot reach
    assert x < 0.0 and abs(u - math.exp(x)) < 0.1 * TIE_WINDOW, (u, x)
    return bs, u, x
