"""Parity criteria for the feedback eq:feed (Section 3) at arbitrary states,
shared by the GPU feedback tests of the orbit, Heun-foot and crown problems.

At every state:
  * the device's Q of its own control agrees with the oracle's Q of the
    oracle's control within one float32 evaluation's tolerance;
  * the device's control attains the oracle's minimum: the oracle, in FP64,
    evaluates Q at the device's (throttle, angle) and finds it within the same
    tolerance of its own minimum.
Away from ties (oracle tie margin >= 1e-4 * max(1, |Q|)), the control itself
agrees on >= 99.9 % of the states: the same throttle and, for thrust, the same
table entry (tabulated search) or an angle within twice the final golden
width (continuous search; where Q is flatter than float32 resolves any angle
of the flat band attains the minimum, which the second check covers)."""
import math

import numpy as np

ANGLE_TOL = 1.2e-3


def _wrapped(du):
    return np.abs((np.asarray(du) + np.pi) % (2 * np.pi) - np.pi)


def table_index(u, K):
    return np.rint((np.asarray(u, dtype=np.float64) + math.pi) * K / (2 * math.pi)).astype(np.int64) % K


def check_feedback(o, V, states, ang_g, thr_g, q_g, tau=None, n_table=None, min_clear=50):
    """o: the oracle; V: the value function both sides read (float64 copy of
    the float32 array); states: n x 4; ang_g/thr_g/q_g: the device's outputs
    (numpy).  n_table: the table size for a tabulated search, None for the
    continuous search.  Returns (states, clear states, thrust states compared)."""
    V = np.asarray(V, dtype=np.float64)
    states = np.asarray(states, dtype=np.float64)
    ao, to, qo, margin = o.feedback(V, states, tau=tau, with_margin=True)
    ang_g = np.asarray(ang_g, dtype=np.float64).reshape(-1)
    thr_g = np.asarray(thr_g).reshape(-1)
    q_g = np.asarray(q_g, dtype=np.float64).reshape(-1)
    scale = np.maximum(1.0, np.abs(qo))
    # one float32 Q: 1e-5*max(1,|Q|) plus the lerps' rounding at the corners' magnitude
    tol = 1e-5 * scale + 1e-6 * np.abs(V).max()
    assert np.all(np.abs(q_g - qo) <= tol), np.max(np.abs(q_g - qo) / tol)
    q_at_dev = np.array([o.q_state(V, y, int(t), float(u), tau) for y, t, u in zip(states, thr_g, ang_g)])
    assert np.all(q_at_dev - qo <= tol), np.max((q_at_dev - qo) / tol)
    clear = margin >= 1e-4 * scale
    same = thr_g == to
    thrust = same & (to == 1)
    if n_table is not None:
        same[thrust] &= table_index(ang_g[thrust], n_table) == table_index(ao[thrust], n_table)
    else:
        same[thrust] &= _wrapped(ang_g[thrust] - ao[thrust]) <= ANGLE_TOL
        # a thrust angle in a band flatter than float32 resolves is a correct answer
        flat = np.zeros_like(same)
        idx = np.flatnonzero(thrust & ~same)
        for c in idx:
            qa = [o.q_state(V, states[c], 1, float(ao[c]) + d, tau) for d in (-ANGLE_TOL, ANGLE_TOL)]
            flat[c] = min(qa) - qo[c] < 1e-5 * scale[c]
        same |= flat
    n_clear = int(clear.sum())
    assert n_clear >= min_clear, n_clear
    if n_clear:
        agree = same[clear].mean()
        assert agree >= 0.999, (agree, np.flatnonzero(clear & ~same)[:8])
    return len(states), n_clear, int((clear & thrust).sum())
