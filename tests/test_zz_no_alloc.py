"""ev_eval_fitness_static: evaluation that allocates nothing (C ABI).

Its results must equal ev_eval_fitness's with device outputs (and the
oracle's), bit for bit, on two calls in a row, the second with a smaller
population; it must take no device block from the context's allocator, and
refuse what does not fit its static array or has no settled plan.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def same_bits(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


def test_static_scratch_evaluation_matches_the_allocating_one():
    import torch

    import paper_1902_09215_amd as ev

    ev.load_library()
    x, y = workloads.cases(48)
    big_sizes = workloads.loguniform_sizes(71, 400, 1, 60000)
    big_buf, big_off = workloads.random_population(71, big_sizes)
    small_buf, small_off = workloads.rhh_population(workloads.SEED_BASE + 1, 100, 2, 6)
    calls = {"alloc": 0}

    def alloc(nbytes, _user):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0)

    def free(ptr, _user):
        torch.cuda.caching_allocator_delete(ptr)

    a = ev.ev_allocator(ev._ALLOC_FN(alloc), ev._FREE_FN(free), None)
    with ev.Context(x, y, allocator=a) as c:
        ev.ev_set_tuning(c.ctx, 1024)  # many work items and slots
        pops = [(c.load(big_buf, big_off), big_buf, big_off), (c.load(small_buf, small_off), small_buf, small_off)]
        for pop, buf, off in pops:  # the larger first, then the smaller
            M = off.size - 1
            want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=8, per_case=True)
            before = calls["alloc"]
            fit = torch.full((M,), -7.0, dtype=torch.float32, device="cuda")
            pc = torch.full((M, 48), -7.0, dtype=torch.float32, device="cuda")
            hits = torch.full((M,), -7, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            ev.ev_eval_fitness_static(c.ctx, pop, fit, 0, pc, hits)
            torch.cuda.synchronize()
            assert calls["alloc"] == before, "the static evaluation took a block from the allocator"
            sf, spc, sh = fit.cpu().numpy(), pc.cpu().numpy(), hits.cpu().numpy()
            # the allocating form, into other device outputs
            fit2 = torch.empty_like(fit)
            pc2 = torch.empty_like(pc)
            hits2 = torch.empty_like(hits)
            torch.cuda.synchronize()
            ev.ev_eval_fitness(c.ctx, pop, 0, out=fit2, out_per_case=pc2, out_hits=hits2)
            torch.cuda.synchronize()
            assert same_bits(sf, fit2.cpu().numpy()).all()
            assert same_bits(spc, pc2.cpu().numpy()).all()
            assert np.array_equal(sh, hits2.cpu().numpy())
            assert same_bits(sf, want_fit).all() and same_bits(spc, want_pc).all()
            assert np.array_equal(sh, oracle.hits(want_pc, y))
        # a population whose result slots do not fit the static array
        huge_sizes = workloads.loguniform_sizes(72, 4000, 10, 1e5)
        hb, ho = workloads.random_population(72, huge_sizes)
        hpop = c.load(hb, ho)
        out = torch.empty(ho.size - 1, dtype=torch.float32, device="cuda")
        with pytest.raises(ev.EvError) as e:
            ev.ev_eval_fitness_static(c.ctx, hpop, out)
        assert e.value.code == ev.EV_ECAP
        # children whose plan's validation verdict is still to be read
        small_pop = pops[1][0]
        c.eval(small_pop)
        kids, _ = ev.ev_generation(c.ctx, small_pop, 3, 0, 2, 10**7)
        kout = torch.empty(100, dtype=torch.float32, device="cuda")
        with pytest.raises(ev.EvError) as e:
            ev.ev_eval_fitness_static(c.ctx, kids, kout)
        assert e.value.code == ev.EV_EINVAL
        kf, _ = c.eval(kids)
        ev.ev_eval_fitness_static(c.ctx, kids, kout)
        torch.cuda.synchronize()
        assert same_bits(kout.cpu().numpy(), kf).all()
