"""The embedded error estimate of one RODAS4 step, from the oracle: the RMS
over the n components of e_k / (atol + rtol max(|y_k|, |ynew_k|)), with e
the embedded error vector (for RODAS4 the last stage vector u_6; Hairer &
Wanner, Sec. VI.4), and the spread of that norm under 1-ulp input changes,
which bounds how far two correct implementations may differ on a cell whose
estimate is dominated by rounding (every component moved by one ulp
either way, one at a time)."""
import numpy as np


def errnorm(om, p, y, h, rtol, atol):
    yo, eo = om.step(p, y, h)
    sc = atol + rtol * np.maximum(np.abs(y), np.abs(yo))
    return float(np.sqrt(np.mean((eo / sc) ** 2))), yo, eo


def errnorm_with_spread(om, p, y, h, rtol, atol):
    """The norm, and its largest change when any one component of y moves by
    one ulp either way (the estimate is a difference of nearly equal stage
    terms, so rounding-level input changes move it well above its own ulp)."""
    en, yo, eo = errnorm(om, p, y, h, rtol, atol)
    spread = 0.0
    for k in range(len(y)):
        for f in (1.0 + 2.0**-52, 1.0 - 2.0**-52):
            y1 = np.array(y, dtype=float)
            y1[k] *= f
            spread = max(spread, abs(errnorm(om, p, y1, h, rtol, atol)[0] - en))
    return en, spread, yo, eo


def errnorm_bar(en_oracle, spread):
    """Allowed |implementation - oracle| for the error norm: 1e-5 relative,
    plus 4x the oracle's own 1-ulp spread, plus an absolute 1e-8.

    The estimate u_6 solves M u_6 = f(Y_6) + sum_j (c_6j / h) u_j, whose
    right-hand side is a difference of nearly equal terms, so two correct
    implementations that round differently (FMA contraction, 1-ulp
    differences of log or 1/x) differ by far more than an ulp of the norm:
    up to 6e-7 relative was seen between the oracle and a host build of the
    device code.  The norm enters the controller only through the accept test
    (<= 1) and 0.9 max(err, 1e-16)^(-1/4) clipped to [0.2, 6]: a 1e-5 relative
    difference moves a step size by 2.5e-6 of itself and can flip a decision
    only for a norm within 1e-5 of 1, while a wrong coefficient or a dropped
    stage changes the norm by an O(1) factor.  The factor 6 of the clip is
    reached for every err below (0.9/6)^4 = 5e-4, so below that the norm
    decides nothing: the norm of a tiny step (1e-6 .. 1e-15, where the
    rounding of the stage terms is a large part of it; 3e-4 relative at 2e-6
    was seen on the GPU) is compared to an absolute 1e-8, which moves a step
    size by at most 5e-6 of itself even at err = 5e-4."""
    return 1e-5 * en_oracle + 4.0 * spread + 1e-8
