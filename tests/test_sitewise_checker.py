"""The per-site draw check used on the reduced-precision GPU form, pinned on
the CPU with the oracle's own draws: an oracle draw passes with no differing
site, and a layer with one site changed to the other state (a planted
mistake) is caught at that site with a margin far outside the tie window."""
import numpy as np

import gpu_helpers as gh
import synth
from oracle import chain as ochain


def test_oracle_draw_passes_and_planted_flip_is_caught():
    Lx, Ly, Lz, z, beta, chi = 5, 4, 3, 1, 0.8, 3
    J = synth.couplings_gauss(Lx, Ly, Lz, 11)
    spins = synth.spins_random(Lx, Ly, Lz, 12)
    margins = []
    rec = ochain.propose(J, spins, z, beta, chi, 2, seed=12345, chain=0, sweep=4, margins=margins)
    lq, bad, worst, closest = gh.sitewise_draw_check(J, spins, z, rec["new"], beta, chi, 2, seed=12345, chain=0,
                                                     sweep=4)
    assert bad == 0 and abs(lq - rec["logq_new"]) < 1e-12 * max(1.0, abs(lq))
    assert abs(closest - min(margins)) < 1e-15
    # flip the site whose uniform is farthest from its threshold
    k = int(np.argmax(margins))
    y, x = divmod(k, Lx)
    planted = rec["new"].copy()
    planted[y, x] = -planted[y, x]
    _, bad, worst, _ = gh.sitewise_draw_check(J, spins, z, planted, beta, chi, 2, seed=12345, chain=0, sweep=4)
    assert bad >= 1 and worst > gh.TIE_REDUCED
