"""pic_step_noalloc (the step for callers that cannot allocate) against
pic_step through the C-ABI: two contexts built from the same inputs, one
stepped by each entry point, must hold bitwise the same particles (matched
by id) and fields, the same integer ledger counts, and fp64 sums equal to
round-off.  Two calls in a row share the fixed scratch array, the second on a
smaller discharge; both cross a compaction (its histograms live in the
array too).  Explicit and implicit cases, with diagnostics sampling."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def P():
    import paper_1310_5284_amd as P
    return P


def pair(wl, tile, sort_every, diag_every):
    a = P().PicContext([wl])
    b = P().PicContext([wl])
    for c in (a, b):
        c.set_schedule(sort_every=sort_every, diag_every=diag_every, tile=tile)
    return a, b


def by_id(ctx):
    st = ctx.state(0)
    out = []
    for sp in st["species"]:
        o = np.argsort(sp["id"], kind="stable")
        out.append({k: v[o] for k, v in sp.items()})
    return st["step"], out


def same_state(a, b):
    # the compaction orders the slots of one bucket by the order in which
    # workgroups reserve them, so particles are matched by id; their values,
    # the integer deposits and everything the FP64 solve makes of them are
    # bitwise equal; the ledger energies and heating sum float32 per-particle
    # terms in groups that depend on which particles a workgroup holds, so
    # they agree to the rounding of those groups: the ledger energies to 1e-8
    # of the kinetic energy (float32 epsilon times the step's work, a small
    # part of it), the heating of a cell, a float32 sum over its particles,
    # to 1e-5 of the largest cell's
    (ta, pa), (tb, pb) = by_id(a), by_id(b)
    assert ta == tb
    for s in range(2):
        for k, v in pa[s].items():
            assert np.array_equal(v, pb[s][k]), (s, k)
    fa, fb = a.fields(0), b.fields(0)
    for k in ("rho", "phi", "E", "chi"):
        assert np.array_equal(fa[k], fb[k]), k
    for s in range(2):
        assert np.array_equal(fa["qfix"][s], fb["qfix"][s])
        assert np.array_equal(fa["cell_count"][s], fb["cell_count"][s])
    la, lb = a.ledger(0), b.ledger(0)
    # every energy term of the step is judged against the kinetic energy
    K = max(np.abs(lb["K_before"]).max(), np.abs(lb["K_after"]).max())
    for k, v in la.items():
        v, w = np.asarray(v), np.asarray(lb[k])
        if v.dtype.kind in "iu":
            assert np.array_equal(v, w), k
        else:
            scale = abs(float(w)) if k == "WE" else K
            np.testing.assert_allclose(v, w, rtol=0, atol=1e-8 * scale, err_msg=k)
    ha, hb = a.heating(0), b.heating(0)
    for s in range(2):
        np.testing.assert_allclose(ha[s], hb[s], rtol=0, atol=1e-5 * np.abs(hb[s]).max())


@pytest.mark.parametrize("scheme", [0, 1])
def test_noalloc_step_equals_pic_step_on_two_calls(scheme):
    big = W.c1(collisions=1, np_per_species=40000 + 77, scheme=scheme)
    small = W.c1(collisions=1, np_per_species=5000 + 13, scheme=scheme)
    small["case"]["seed"] = 0x5A11
    a, b = pair(big, tile=1024, sort_every=16, diag_every=3)
    a.step_noalloc(40)
    b.step(40)
    same_state(a, b)
    c, d = pair(small, tile=1024, sort_every=16, diag_every=3)
    c.step_noalloc(40)
    d.step(40)
    same_state(c, d)
    for x in (a, b, c, d):
        x.close()


def test_noalloc_step_rejects_a_schedule_beyond_the_array():
    # 16 cases of 1e5 particles per species at tile 256: about 15 600
    # particle-pass workgroups, more than the ~12 700 rows the array holds
    wls = [W.c1(collisions=1, np_per_species=100000) for _ in range(16)]
    ctx = P().PicContext(wls)
    ctx.set_schedule(sort_every=64, diag_every=0, tile=256)
    with pytest.raises(Exception, match="scratch"):
        ctx.step_noalloc(1)
    ctx.close()
