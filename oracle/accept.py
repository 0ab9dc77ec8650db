"""Independence Metropolis chain over tensor-network proposals (Sec. II, Eq. (3); Appendix A).

Proposals are drawn independently of the current state, so g(s'|s) = q(s') and Eq. (3) becomes

    p_a(s'|s) = min{1, [q(s) / q(s')] [P(s') / P(s)]} = min{1, exp(Delta)},
    Delta = (-beta E(s') - log q(s')) - (-beta E(s) - log q(s)),

as in the periodic-chain example of Appendix A.  Readings where the paper is silent: the first
proposal of a chain initialises it unconditionally (independent proposals need no burn-in); a
proposal is accepted iff Delta >= 0 or u < exp(Delta) (strict), with u the 53-bit Philox uniform
number ``step`` of the stream keyed (seed, STREAM_ACCEPT) with counter words
(chain, realization, 0); one uniform is consumed per step whether or not it is needed.

This is test infrastructure (see the package docstring).
"""
import math

import numpy as np

from . import philox


def accept_uniforms(seed, realization, chain, steps):
    return philox.uniforms((seed, philox.STREAM_ACCEPT), np.asarray(steps, dtype=np.uint64),
                           c1=chain, c2=realization, c3=0)


def chain(E_prop, logq_prop, beta, seed=0, realization=0, chain_index=0, first_step=0,
          state=None):
    """Run one chain over proposals in order.

    E_prop, logq_prop : (K,) energies and log q of the proposals
    state             : None (uninitialised) or dict(idx, E, logq) of the current state, where
                        idx = -1 refers to a configuration from an earlier batch
    returns dict: accepted (K,) bool (the initialising step counts as not accepted), current
    (K,) index of the chain's configuration after each step (-1 = from an earlier batch),
    init (K,) bool marking the initialising step, and the final state.
    """
    K = len(E_prop)
    u = accept_uniforms(seed, realization, chain_index, first_step + np.arange(K))
    accepted = np.zeros(K, dtype=bool)
    init = np.zeros(K, dtype=bool)
    current = np.zeros(K, dtype=np.int64)
    st = None if state is None else dict(state)
    for k in range(K):
        Ek, lk = int(E_prop[k]), float(logq_prop[k])
        if st is None:
            st = {"idx": k, "E": Ek, "logq": lk}
            init[k] = True
        else:
            delta = (-beta * Ek - lk) - (-beta * st["E"] - st["logq"])
            if delta >= 0.0 or u[k] < math.exp(delta):
                st = {"idx": k, "E": Ek, "logq": lk}
                accepted[k] = True
        current[k] = st["idx"]
    out_state = dict(st)
    out_state["idx"] = -1
    return {"accepted": accepted, "current": current, "init": init, "state": out_state}
