"""Per-cell heating (the field work of a step attributed to the cell a particle
starts the step in) against the oracle, teacher-forced one step at a time.

Sampled every step (diagnostics every step), so the accumulator's increase
over a step is that step's heating profile; the oracle, loaded with the GPU
state of the step, computes the same profile in FP64.  The m = 2 weighting
runs here on purpose: its deposit touches node N, one past the last cell of
the heating profile, and the profile must stay within its N cells.  Cell
counts with N % 4 == 0 and != 0 put the end of the profile at different
alignments."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import to_oracle_species

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_cells", [64, 66])
@pytest.mark.parametrize("scheme", [0, 1])
def test_heating_profile_per_cell_matches_oracle(n_cells, scheme):
    import paper_1310_5284_amd as P
    wl = W.ccp_workload("ccp_heating", n_cells=n_cells, np_per_species=8192 + 33,
                        volts=100.0, p_mtorr=50.0, scheme=scheme, collisions=1,
                        seed=0x4EA7 + n_cells, gather=2,
                        dt=1.0 / ((400.0 if scheme == 0 else 100.0) * 13.56e6))
    ctx = P.PicContext([wl])
    ctx.set_schedule(sort_every=16, diag_every=1, tile=1024)
    worst = 0.0
    for n in range(12):
        h0 = ctx.heating(0)
        st = ctx.state(0)
        sim = oracle.Sim(dict(wl["case"], step0=st["step"]), to_oracle_species(st, wl),
                         wl["processes"], startup=False)
        sim.step(1)
        ctx.step(1)
        h1 = ctx.heating(0)
        he, hi = sim.heating()
        for s, ho in enumerate((he, hi)):
            hg = h1[s] - h0[s]
            assert hg.shape == (n_cells,)
            assert np.all(np.isfinite(hg))
            scale = np.abs(ho).max()
            if scale == 0.0:
                assert np.abs(hg).max() == 0.0
                continue
            # each particle's work in float32, summed per cell: ~1e-6 of the
            # largest cell's heating
            err = float(np.abs(hg - ho).max() / scale)
            worst = max(worst, err)
            assert err <= 1e-4, (n, s, err)
            # the total is the step's field work of the ledger
            assert abs(hg.sum() - sim.ledger()["work"][s]) <= 1e-4 * np.abs(ho).sum()
    print("worst per-cell heating error", worst)
    ctx.close()
