"""Parity tolerances for full sums, derived from the arithmetic.

Every term t_Z = (-1)^(n-|Z|) / sqrt(det (I-O)_Z) is formed by one
backward-stable factorisation on each side (GPU and oracle), in different
orders, so its relative rounding error is a sum of many independent
roundings: small, of either sign, and independent between subsets and
between the two sides.  Both sides add their terms without further error
(double-double on the GPU, __float128 in the oracle).  With a per-term
relative error of standard deviation at most RHO * u on a side of unit
roundoff u, the difference of two full sums has standard deviation at most

    RHO * sqrt(u_gpu^2 + u_oracle^2) * sqrt(sum_Z t_Z^2),

and the tests allow SIGMAS of them.  This is the Sec. 5 view of fidelity
(the relative difference of two evaluations) with the cancellation made
explicit: relative to |Tor| the bound grows like R = sum|t| / |Tor| divided
by about sqrt(2^n).

RHO is taken above what the measurements show: for the workloads here the
spread of the FP64 terms' errors is below one unit of roundoff per term
(n = 20 against __float128, n = 24 and 30 against the extended-precision
oracle).  A worst-case bound (c n kappa u sum|t|) would instead exceed |Tor|
itself at n >= 24 and could not fail.
"""
import math

U64 = 2.0 ** -53     # FP64
ULD = 2.0 ** -64     # x87 extended (the oracle's "ld" mode)
UQ = 2.0 ** -113     # __float128
UDD = 2.0 ** -100    # the double-double factor: a few units of 2^-104 per step
RHO = 4.0
SIGMAS = 6.0


def sum_bound(sum_sq, *units):
    """Allowed |A - B| between two full sums whose sides round each term with
    the given unit roundoffs."""
    return SIGMAS * RHO * math.sqrt(sum(u * u for u in units)) * math.sqrt(sum_sq)


UNIT_OF_MODE = {"f64": U64, "ld": ULD, "quad": UQ}
