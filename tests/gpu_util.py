"""Helpers shared by the GPU tests: device tensors from numpy, and a pair of
maps (HIP library + oracle) fed the same seeded inputs and PRF key."""
import numpy as np

import oracle as O
import synth


def dev_u64(a):
    import torch

    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64).copy()).cuda()


def dev_u8(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8).copy()).cuda()


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


class Twin:
    """A GPU map and an oracle map with the same parameters and key."""

    def __init__(self, cap, vs, key=bytes(range(32)), trace=True, observable=0, flags=0, seal=False,
                 decomposed=False, **kw):
        import paper_2509_01742_amd as B

        okw = {}
        for a, b in (("c", "c"), ("alpha_permille", "alpha_pm"), ("bin_slots", "bin_slots"), ("pm_choices", "d"),
                     ("pm_keys_per_row", "kpr"), ("pm_row_slots", "W")):
            if a in kw:
                okw[b] = kw[a]
        self.p = B.params(cap, vs, key=key, observable=observable, **kw)
        # a sealed twin shares its fixed key with the oracle: a test-only reuse of the page key
        self.p.flags |= (B.BOLT_F_TRACE if trace else 0) | flags | (
            (B.BOLT_F_SEAL | B.BOLT_F_SEAL_KEY_REUSE) if seal else 0) | (B.BOLT_F_DECOMPOSED if decomposed else 0)
        self.g = B.Map(self.p)
        self.o = O.OracleMap(cap, vs, key=key, trace=trace, seal=seal, decomposed=decomposed, **okw)
        self.seal = seal
        self.vs = vs
        self.B = B

    def build(self, keys, vals, mode=0):
        import torch

        rc_o = self.o.build(keys, vals, mode)
        rc_g = self.g.build(dev_u64(keys) if len(keys) else None, dev_u8(vals) if len(keys) else None)
        torch.cuda.synchronize()
        return rc_o, rc_g, self.g.status()

    def access(self, ops, keys, vals_in):
        import torch

        q = len(ops)
        rc_o, vo_o, st_o = self.o.access(ops, keys, vals_in)
        d_ops, d_keys, d_vin = dev_u8(ops), dev_u64(keys), dev_u8(vals_in)
        d_vout = torch.zeros((q, self.vs), dtype=torch.uint8, device="cuda")
        d_st = torch.zeros(q, dtype=torch.uint8, device="cuda")
        rc_g = self.g.access(d_ops, d_keys, d_vin, d_vout, d_st)
        torch.cuda.synchronize()
        return (rc_o, vo_o, st_o), (rc_g, self.g.status(), d_vout.cpu().numpy(), d_st.cpu().numpy())

    def assert_same_state(self, trace=True):
        g, o = self.g, self.o
        assert np.array_equal(g.observable(), o.observable()), "observable pages differ"
        if self.seal:
            assert np.array_equal(g.tags(), o.tags()), "page tags differ"
            assert np.array_equal(g.versions(), o.versions()), "page write counts differ"
        assert np.array_equal(g.hbm_bins(), o.hbm_bins()), "HBM bins differ"
        assert np.array_equal(g.loads(), o.loads()), "bin loads differ"
        assert g.stash() == o.stash(), "stash differs"
        assert g.pmap() == o.pmap(), "position map differs"
        st = g.stats()
        assert st["live"] == o.live and st["steps"] == o.ctr
        assert st["stash_live"] == o.stash_live
        if trace:
            tg, to = g.trace(), o.trace()
            assert tg.size == to.size, (tg.size, to.size)
            assert np.array_equal(tg, to), "trace differs"


def workload(n, vs, seed):
    return synth.keys(n, seed), synth.values(n, vs, seed + 1)
