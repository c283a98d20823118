"""Shared helpers of the GPU parity tests: drive the HIP library (through the
C ABI binding) and the CPU oracle over the same seeded inputs and compare
everything the method fixes: C_t bit for bit, R_t, the sweep trace (moves and
exact Delta N of every sweep of every level), the exact numerator N and 2m."""
import numpy as np

from oracle import oracle as O
from paper_1904_08553_amd import dc

MODES = {"delta": (O.MODE_DELTA, dc.MODE_DELTA), "all": (O.MODE_ALL, dc.MODE_ALL),
         "static": (O.MODE_STATIC, dc.MODE_STATIC)}


def make_pair(n, u, v, w, mode="delta", max_levels=32, max_sweeps=100, guard=1,
              del_rule=0, tau_den=1_000_000, cascade=None, slm=False):
    """The oracle and the GPU library on the same graph and options (slm:
    the smart local moving levels instead of Louvain's)."""
    om, gm = MODES[mode]
    o = O.Oracle(n, u, v, w, mode=om, max_levels=max_levels, max_sweeps=max_sweeps,
                 singleton_guard=guard, del_rule=del_rule, tau_den=tau_den, cascade=cascade,
                 algorithm=O.ALGO_SLM if slm else O.ALGO_LOUVAIN)
    g = dc.DynamicCommunities(n, u, v, w, mode=gm, max_levels=max_levels,
                              max_sweeps=max_sweeps, singleton_guard=guard, del_rule=del_rule,
                              tau_den=tau_den, cascade=cascade,
                              algorithm=dc.ALGO_SLM if slm else dc.ALGO_LOUVAIN)
    return o, g


def compare(o, g, where, check_R=True):
    Cg = g.communities()
    assert np.array_equal(o.C, Cg), f"{where}: C differs at {np.flatnonzero(o.C != Cg)[:10]}"
    if check_R:
        Rg = g.last_R()
        assert np.array_equal(o.R.astype(np.uint8), Rg), f"{where}: R_t differs"
    tg = g.last_trace()
    assert tg == o.trace, f"{where}: sweep trace differs\noracle {o.trace[:8]}\ngpu    {tg[:8]}"
    st = g.last_stats()
    assert (st.N, st.two_m) == (o.info.N, o.info.two_m), f"{where}: N/2m differ"
    q, N, tm = g.modularity()
    qo, No, tmo = o.modularity()
    assert (N, tm) == (No, tmo), f"{where}: modularity numerator differs"
    assert abs(q - qo) <= 1e-9 * max(1.0, abs(qo))


def step_pair(o, g, b):
    o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
