"""The OpenMP build of the oracle (the same source; its pragmas spread the
pencils of each sweep, the primitive conversion and the source loop over
threads, every one writing its own cells) gives bitwise the plain build's
right-hand sides and runs, on every boundary kind, model, reconstruction and
grid kind, and reports non-physical states the same way."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2305_09163_amd import workloads as W


def cases():
    bub, wb = W.bubble_collapse_3d(n=(17, 15, 19))
    yield "bubble_extrap", bub, wb, oracle.RECON_WENO5
    yield "bubble_cbc_mixed", dataclasses.replace(bub, bc=(2, 0, 1, 1, 2, 2)), wb, oracle.RECON_WENO5
    yield "bubble_kapila", dataclasses.replace(bub, model=1), wb, oracle.RECON_WENO5
    yield "bubble_weno3", bub, wb, oracle.RECON_WENO3
    sp, ws = W.random_smooth_periodic(2, 33)
    yield "smooth_2d", sp, ws, oracle.RECON_FIRST
    st, wst = W.bubble_collapse_3d(n=16, stretch=0.5)
    yield "stretched_3d", st, wst, oracle.RECON_WENO5


@pytest.mark.parametrize("name,spec,w,recon", list(cases()), ids=[c[0] for c in cases()])
def test_threaded_oracle_is_bitwise_plain(name, spec, w, recon):
    q = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    r1, s1 = oracle.rhs(spec, q, recon=recon)
    q1, t1, u1 = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 3, cfl=0.3, recon=recon)
    with oracle.threaded() as n:
        assert n >= 1
        r2, s2 = oracle.rhs(spec, q, recon=recon)
        q2, t2, u2 = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 3, cfl=0.3, recon=recon)
    assert s1 == s2 == oracle.OK and u1 == u2 == oracle.OK
    assert np.array_equal(r1, r2) and np.array_equal(q1, q2) and t1 == t2


def test_threaded_oracle_flags_nonphysical_states():
    spec, w = W.bubble_collapse_3d(n=12)
    q = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    q[0, 6, 6, 6] = -1.0   # negative partial density in one interior cell
    q[1, 6, 6, 6] = -1.0
    _, s1 = oracle.rhs(spec, q)
    with oracle.threaded():
        _, s2 = oracle.rhs(spec, q)
    assert s1 == s2 == oracle.E_NONPHYSICAL
