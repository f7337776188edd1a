"""The GPU's realisation of null-collision candidacy (Sec. III, MCC) against
the law it must follow and against the oracle's uncapped waits.

Every particle is a candidate in every step with probability P_null,
independently.  The kernels realise this with geometric waiting times packed
into 17 bits of the cell word: a wait beyond the count range is stored as the
largest count with a capped flag, and when such a count runs out the trial of
that step is drawn afresh (draw 4 of the step's stream; the geometric law is
memoryless).  The oracle holds its waits uncapped, so:
  * a first wait equals the oracle's, or is capped exactly when the oracle's
    exceeds the count range (low P_null, where both kinds occur);
  * an expiring capped count makes the particle a candidate at rate P_null,
    and leaves a wait that is again Geo0(P_null) -- checked in law and, per
    particle, against the oracle's draws of the same stream.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

WAIT_MAX = 0x1FFFF
WAIT_CAPPED = 0x20000


def P():
    import paper_1310_5284_amd as P
    return P


def encode(w):
    w = np.asarray(w, dtype=np.int64)
    return np.where(w > WAIT_MAX, WAIT_MAX | WAIT_CAPPED, w).astype(np.int64)


def oracle_sim(wl):
    case, sps, procs = W.to_oracle(wl)
    return oracle.Sim(case, sps, procs)


def test_first_waits_match_the_uncapped_oracle_at_low_pnull():
    # P_null ~ 2e-5: a few % of the first waits exceed 2^17 - 1
    wl = W.c1(collisions=1, np_per_species=60000)
    wl["case"]["gas_density_m3"] = W.gas_density(50.0) * 2.8e-5
    sim = oracle_sim(wl)
    p = 1.0 - math.exp(-sim.numax(0) * wl["case"]["dt_s"])
    assert 5e-6 < p < 5e-5
    ctx = P().PicContext([wl])
    st = ctx.state(0)
    words = st["species"][0]["mcc_wait"].astype(np.int64)
    ids = st["species"][0]["id"]
    ow = np.array([sim.first_wait(0, int(i), 0) for i in ids], dtype=np.int64)
    capped = (words & WAIT_CAPPED) != 0
    n = ids.size
    q = (1.0 - p) ** (WAIT_MAX + 1)
    assert abs(capped.sum() - n * q) <= 5 * math.sqrt(n * q * (1 - q)), (capped.sum(), n * q)
    # per particle: the same draw, stored whole or capped
    bad = int((encode(ow) != words).sum())
    print("p", p, "capped", int(capped.sum()), "of", n, "mismatched", bad)
    assert bad <= 2
    ctx.close()


def test_expiring_capped_wait_is_an_open_trial():
    # every particle loaded with a capped count of 2: no candidates in steps 0
    # and 1, then each one's trial of step 2 is drawn afresh
    wl = W.c1(collisions=1, np_per_species=200000)
    for sp in wl["species"]:
        sp["mcc_wait"] = np.full(sp["cell"].size, WAIT_CAPPED | 2, np.uint32)
    sim = oracle_sim(wl)
    pn = [1.0 - math.exp(-sim.numax(s) * wl["case"]["dt_s"]) for s in range(2)]
    ctx = P().PicContext([wl])
    ctx.set_schedule(sort_every=64, diag_every=0, tile=4096)
    for step in range(2):
        ctx.step(1)
        assert list(ctx.ledger(0)["n_candidates"]) == [0, 0], step
    n_live = ctx.counts(0)["n"]
    ctx.step(1)
    led = ctx.ledger(0)
    st = ctx.state(0)
    for s in range(2):
        n, p = n_live[s], pn[s]
        c = int(led["n_candidates"][s])
        sd = math.sqrt(n * p * (1 - p))
        print("species", s, "P_null", p, "candidates", c, "expected", n * p)
        assert abs(c - n * p) <= 5 * sd + 1
        sp = st["species"][s]
        words = sp["mcc_wait"].astype(np.int64)
        # a capped word left by this step is a fresh draw at the full count
        assert not np.any(((words & WAIT_CAPPED) != 0) & ((words & WAIT_MAX) != WAIT_MAX))
        # the waits left are Geo0(P_null) again (memoryless): mean and P(0)
        w = np.where(words & WAIT_CAPPED, WAIT_MAX + 1, words & WAIT_MAX).astype(np.float64)
        m = w.size
        mean, sdm = (1 - p) / p, math.sqrt(1 - p) / p / math.sqrt(m)
        if p > 1e-3:
            assert abs(w.mean() - mean) <= 5 * sdm, (w.mean(), mean)
            z = (w == 0).mean()
            assert abs(z - p) <= 5 * math.sqrt(p * (1 - p) / m) + 1.0 / m
        # per particle, from the same stream: the open trial is candidacy
        # iff draw 4 of step 2 gives W = 0; a candidate then draws its next
        # wait from draw 0, a non-candidate keeps W - 1
        sample = np.arange(0, sp["id"].size, max(1, sp["id"].size // 4000))
        bad = 0
        for k in sample:
            pid = int(sp["id"][k])
            W4 = sim.first_wait(s, pid, 2)
            if W4 == 0:
                exp = sim.wait_step(s, pid, 2, 0)[1]
            else:
                exp = W4 - 1
            bad += int(encode(exp) != words[k])
        print("species", s, "sampled", sample.size, "mismatched", bad)
        assert bad <= 2
    ctx.close()
