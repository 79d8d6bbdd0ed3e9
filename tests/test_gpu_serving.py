"""Ensemble serving on the GPU: continuous batching of independent domains.

A served job's result must equal the single-domain step of the same domain
bit for bit (the batched launches run the single-domain device code on each
job's data), and so must be the same alone and in any mix.  The single-domain
path itself is checked against the FP64 oracle by the parity tests; one case
here also compares a served FP64 job with the oracle directly."""
import numpy as np
import pytest

from paper_2512_04997_amd import workloads as W
from tests.parity import TOL, pop_err, vec_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def _jobs(prec="fp32"):
    """Uneven jobs: ragged tiles in every axis, settling and shear, a
    fluid-only job with the TRT operator, one with three solids per cell, and
    different step counts."""
    rng = W.SplitMix64(77)
    out = []
    cfg, parts = W.serving_job(rng, "settle", 32, 0.62, 12, precision=prec)
    out.append((cfg, parts, 7))
    box = (72, 42, 38)
    bc = ["periodic"] * 4 + ["moving"] * 2
    wu = [[0.0] * 3 for _ in range(6)]
    wu[4] = [-0.02, 0.0, 0.0]
    wu[5] = [0.02, 0.0, 0.0]
    radii = 3.0 + 3.0 * rng.uniform(25)
    pos = W.rsa_spheres(rng, 25, radii, box, [True, True, False])
    cfg = W.base_config(box, 0.85, bc=bc, wall_u=wu, precision=prec)
    out.append((cfg, W.spheres(pos, radii[:len(pos)], 1.5), 5))
    cfg = W.base_config((48, 22, 26), 0.7, precision=prec, bc=["periodic"] * 4 + ["noslip"] * 2,
                        body_force=[2e-6, 0.0, 0.0], collision="trt")
    out.append((cfg, None, 6))
    cfg, parts = W.serving_job(rng, "shear", 32, 0.58, 10, precision=prec)
    cfg["max_solids"] = 3
    out.append((cfg, parts, 4))
    return out


def _state(D):
    P = D.particles() if D.np else {}
    return D.populations(), P


def _same(a, b):
    fa, Pa = a
    fb, Pb = b
    assert np.array_equal(fa, fb), float(np.max(np.abs(fa - fb)))
    for k in Pa:
        assert np.array_equal(Pa[k], Pb[k]), (k, float(np.max(np.abs(Pa[k] - Pb[k]))))


def _single(ps, cfg, parts, steps):
    D = ps.Domain(cfg, parts)
    D.step(steps)
    D.sync()
    s = _state(D)
    D.close()
    return s


def _serve(ps, jobs, max_jobs, stagger=0, budget=0):
    """A serving loop: job k is submitted after k*stagger iterations; a done
    job is read and released at once.  Returns states, infos and release
    times in job order."""
    S = ps.Server(max_jobs=max_jobs, hbm_budget=budget, precision=jobs[0][0]["precision"])
    ids, states, infos, released = [], {}, {}, {}
    it = 0
    pending = list(jobs)
    while pending or len(states) < len(ids):
        while pending and it >= len(ids) * stagger:
            cfg, parts, steps = pending.pop(0)
            ids.append(S.submit(cfg, parts, steps))
        n_active, _ = S.iterate()
        it += 1
        if n_active == 0:
            S.drain()
        for j in ids:
            if j in states:
                continue
            info = S.job(j)
            assert info["state"] != "failed", info
            if info["state"] == "done":
                states[j] = _state(S.domain(j))
                infos[j] = info
                S.release(j)
                released[j] = ps.clock()
        assert it < 2000
    S.close()
    return [states[j] for j in ids], [infos[j] for j in ids], [released[j] for j in ids]


def test_served_jobs_equal_single_domain_steps(ps):
    jobs = _jobs()
    ref = [_single(ps, *j) for j in jobs]
    got, infos, _ = _serve(ps, jobs, max_jobs=4, stagger=2)
    for k in range(len(jobs)):
        assert infos[k]["state"] == "done" and infos[k]["steps_done"] == jobs[k][2]
        _same(got[k], ref[k])


def test_alone_equals_in_the_mix(ps):
    jobs = _jobs()
    mix, _, _ = _serve(ps, jobs, max_jobs=3, stagger=1)
    for k in (0, 1):
        alone, _, _ = _serve(ps, [jobs[k]], max_jobs=1)
        _same(alone[0], mix[k])


def test_admission_respects_slots_and_budget(ps):
    jobs = _jobs()
    fps = [ps.footprint(c, p) for c, p, _ in jobs]
    budget = max(fps) + min(fps) // 2
    _, infos, rel = _serve(ps, jobs, max_jobs=4, budget=budget)
    # a job holds its memory from admission to release; two jobs held at once
    # must fit the budget together
    for a in range(len(jobs)):
        assert infos[a]["footprint"] == fps[a]
        for b in range(a + 1, len(jobs)):
            if infos[a]["t_admit"] < rel[b] and infos[b]["t_admit"] < rel[a]:
                assert fps[a] + fps[b] <= budget
    # one slot: jobs are admitted one after the other, in arrival order
    _, infos1, _ = _serve(ps, jobs, max_jobs=1)
    for a in range(1, len(jobs)):
        assert infos1[a]["t_admit"] >= infos1[a - 1]["t_admit"]


def test_footprint_is_the_allocation(ps):
    for cfg, parts, _ in _jobs():
        D = ps.Domain(cfg, parts)
        assert D.info()["device_bytes"] == ps.footprint(cfg, parts)
        D.close()


def test_served_fp64_job_matches_oracle(ps, oracle_mod):
    cfg, parts, _ = _jobs("fp64")[0]
    steps = 3
    states, _, _ = _serve(ps, [(cfg, parts, steps)], max_jobs=2)
    O = oracle_mod.OracleDomain(cfg, parts)
    O.step(steps)
    f, P = states[0]
    assert pop_err(f, O.populations()) < TOL["fp64"]
    Po = O.particles()
    assert vec_err(P["pos"], Po["pos"]) < TOL["fp64"]
    assert vec_err(P["vel"], Po["vel"]) < TOL["fp64"]


def test_rejects_jobs_it_cannot_batch(ps):
    S = ps.Server(max_jobs=2, precision="fp32")
    cfg = W.base_config((32, 32, 32), 0.7, precision="fp64")
    with pytest.raises(ps.PsmdemError):
        S.submit(cfg, None, 10)  # precision differs
    cfg = W.base_config((1024, 128, 128), 0.7, precision="fp32")
    with pytest.raises(ps.PsmdemError):
        S.submit(cfg, None, 10)  # 16384 tiles
    cfg = W.base_config((32, 32, 32), 0.7, precision="fp32")
    j = S.submit(cfg, None, 0)
    S.iterate()
    S.drain()
    assert S.job(j)["state"] == "done"
    S.release(j)
    S.close()


def test_rejects_a_job_larger_than_the_budget(ps):
    """A job whose footprint alone exceeds the HBM budget is refused with
    PSMDEM_E_INVALID at submission; one that fits is admitted and runs."""
    small = W.base_config((32, 32, 32), 0.7, precision="fp32")
    big = W.base_config((128, 128, 128), 0.7, precision="fp32")
    fs, fb = ps.footprint(small), ps.footprint(big)
    assert fb > 4 * fs
    S = ps.Server(max_jobs=2, hbm_budget=2 * fs, precision="fp32")
    with pytest.raises(ps.PsmdemError) as e:
        S.submit(big, None, 5)
    assert e.value.code == ps.E_INVALID
    j = S.submit(small, None, 3)
    for _ in range(20):
        n_active, n_queued = S.iterate()
        if n_active == 0 and n_queued == 0:
            break
    S.drain()
    assert S.job(j)["state"] == "done" and S.job(j)["footprint"] == fs
    S.release(j)
    S.close()

