"""Lockstep harness shared by the GPU parity tests: a libpsl walk and an
oracle walk stepped together through Algorithm 1, compared after every step,
with steps flagged ambiguous resolved by the oracle's decision."""
import numpy as np

import oracle

F_RTOL = 1e-12
MARGIN = 5e-13


AMBIG = oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE


def _gpu_ambig(flags):
    """The oracle's ambiguity bits for a walk's PSL_STEP_* flags."""
    from paper_2107_09801_amd import libpsl
    return ((oracle.AMBIG_ARGMIN if flags & libpsl.STEP_AMBIG_ARGMIN else 0) |
            (oracle.AMBIG_COMPARE if flags & libpsl.STEP_AMBIG_COMPARE else 0))


def _near_edge(x, edge, scale, tol=1e-11):
    return abs(abs(x) - edge) <= tol * scale


def _flags_agree(g_amb, tr, ow, vl_before, margin):
    """The GPU's ambiguity bits equal the oracle's, except where a value lies
    so close to the edge of the margin window that the 1e-12 agreement of F
    decides on which side it falls."""
    if g_amb == tr["flags"] & AMBIG:
        return True
    diff = g_amb ^ (tr["flags"] & AMBIG)
    if diff & oracle.AMBIG_ARGMIN:
        F, _ = ow.last_neighbourhood()
        thr = tr["F_min"] * (1 + oracle.TAU)
        if not np.any(np.abs(np.abs(F - thr) - margin * tr["F_min"]) <= 1e-11 * tr["F_min"]):
            return False
    if diff & oracle.AMBIG_COMPARE:
        v = tr["value_step"]
        ok = any(_near_edge(v - e, margin * vl_before, vl_before)
                 for e in (vl_before * (1 - oracle.TAU), vl_before * (1 + oracle.TAU)))
        if not ok:
            return False
    return True


def impose_oracle_state(ctx, w, ow):
    """Overwrite the GPU walk with the oracle walk's state (a flagged step is
    resolved by the oracle's tie rule): its scalars and its three sequences;
    the library recomputes C, C of the local best and the pivot's F and PSL
    from the bits."""
    ck = ctx.checkpoint(w)
    o = ow.read()
    st = ck["state"]
    st.alpha, st.value_local, st.psl_best = o["alpha"], o["value_local"], o["psl_best"]
    st.unimproved, st.t, st.q = o["unimproved"], o["t"], o["q"]
    ctx.restore(w, {"state": st, "pivot": o["pivot"], "local_best": o["local_best"], "best": o["best"]})


def run_lockstep(ctx, w, ow, steps, check_every=1, margin=MARGIN):
    """Step the GPU walk and the oracle walk together. Every step compares the
    start, the move, F of the move, psl_best, alpha, unimproved and v_local,
    and (every check_every steps) the pivot, C, local best and best sequence.
    A step either side flags ambiguous must carry the same flags on both
    sides; it is then resolved by imposing the oracle's state on the GPU walk
    and the walk goes on. Returns (steps compared, steps imposed)."""
    compared = imposed = 0
    for t in range(steps):
        vl_before = ow.read()["value_local"]
        ctx.step_batch([w], 1)
        tr = ow.step()
        g = ctx.read_walk(w, bits=(t % check_every == 0), C=(t % check_every == 0))
        assert g["last_start"] == tr["start"], t
        g_amb = _gpu_ambig(g["last_flags"])
        if g_amb or tr["flags"] & AMBIG:
            assert _flags_agree(g_amb, tr, ow, vl_before, margin), (t, g["last_flags"], tr["flags"])
            impose_oracle_state(ctx, w, ow)
            g = ctx.read_walk(w)
            o = ow.read()
            for key in ("pivot", "C", "local_best", "best"):
                assert np.array_equal(g[key], o[key]), (t, key)
            assert g["t"] == o["t"] and g["psl_best"] == o["psl_best"] and g["alpha"] == o["alpha"]
            imposed += 1
            continue
        assert g["last_k"] == tr["k"], t
        assert abs(g["last_value_step"] - tr["value_step"]) <= F_RTOL * tr["value_step"], t
        assert g["psl_best"] == tr["psl_best"] and g["alpha"] == tr["alpha"], t
        assert g["unimproved"] == tr["unimproved"] and g["t"] == t + 1, t
        assert abs(g["value_local"] - tr["value_local"]) <= F_RTOL * tr["value_local"], t
        if t % check_every == 0:
            o = ow.read()
            assert np.array_equal(g["pivot"], o["pivot"]), t
            assert np.array_equal(g["C"], o["C"]), t
            assert np.array_equal(g["local_best"], o["local_best"]), t
            assert np.array_equal(g["best"], o["best"]), t
        compared += 1
    return compared, imposed
