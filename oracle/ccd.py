"""One coordinate update of cyclic coordinate descent (Secs. 2.3-2.4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The objective maximised along coordinate j is g(beta_j) = l(beta_j) +
pi(beta_j), with the l1 penalty pi = -gamma |beta_j| or the l2 penalty
pi = -beta_j^2 / (2 tau) (Sec. 2.3).  The step is the one-dimensional
Newton step -g'/g'' of the penalised objective (Sec. 2.4), then limited by
the trust region: beta_j += sgn(step) min(|step|, Delta_j) and
Delta_j <- max(2 |step|, Delta_j / 2), starting from Delta_j = 1.

l1 at beta_j = 0 (Sec. 2.4, directional derivatives): the derivative of g
is g' - gamma in the positive direction and g' + gamma in the negative one;
move only in a direction in which the objective increases, else stay at 0.

Readings where the paper is silent:
  * l1 with beta_j != 0: an l1 Newton step that would carry beta_j across
    zero stops at zero (the step becomes -beta_j), as in the coordinate
    descent of Genkin et al. that the paper follows;
  * the trust-region width is updated from the Newton step before the
    trust-region clip (the paper reuses the symbol of the unclipped step);
  * a penalised second derivative that is not strictly negative (e.g. an
    all-zero or constant column without l2 penalty) gives a zero step.
"""
import math

PENALTY_NONE = 0
PENALTY_L1 = 1
PENALTY_L2 = 2


def newton_step(g1, g2, beta_j, penalty, lam):
    """The penalised Newton step of Sec. 2.4 (before the trust region)."""
    if penalty == PENALTY_NONE:
        return -g1 / g2 if g2 < 0 else 0.0
    if penalty == PENALTY_L2:
        tau = lam
        d1 = g1 - beta_j / tau
        d2 = g2 - 1.0 / tau
        return -d1 / d2 if d2 < 0 else 0.0
    if penalty == PENALTY_L1:
        gamma = lam
        if not g2 < 0:
            return 0.0
        if beta_j != 0.0:
            s = 1.0 if beta_j > 0 else -1.0
            step = -(g1 - gamma * s) / g2
            if (beta_j + step) * s < 0:       # would cross zero: stop at it
                step = -beta_j
            return step
        if g1 - gamma > 0:                   # objective rises towards +
            return -(g1 - gamma) / g2
        if g1 + gamma < 0:                   # objective rises towards -
            return -(g1 + gamma) / g2
        return 0.0
    raise ValueError(penalty)


def update(g1, g2, beta_j, delta_j, penalty, lam):
    """Return (new beta_j, new Delta_j, applied step)."""
    step = newton_step(g1, g2, beta_j, penalty, lam)
    applied = math.copysign(min(abs(step), delta_j), step) if step != 0 else 0.0
    new_delta = max(2.0 * abs(step), delta_j / 2.0)
    return beta_j + applied, new_delta, applied


def penalty_value(beta, penalty, lam):
    """pi(beta) of Sec. 2.3 (a non-positive number)."""
    if penalty == PENALTY_NONE:
        return 0.0
    if penalty == PENALTY_L1:
        return -lam * sum(abs(b) for b in beta)
    if penalty == PENALTY_L2:
        return -sum(b * b for b in beta) / (2.0 * lam)
    raise ValueError(penalty)
