"""HBPC(q, k_max) time step: Algorithm 1 (Sec. 2.1) over abstract operators.

One step from w^n (= w_1, held fixed through the step):

Predict (Eq. predictor, written as Eq. Newton_Residual with Eq.
nonlinear_predictor): for l = 2..s, with dc = c_l - c_{l-1},
alpha1 = dc/2, alpha2 = dc^2/6, solve
    W - alpha1 dt R1(W) + alpha2 dt^2/2 R2(W) = b,
    b = w_{l-1} + alpha1 dt R1(w_{l-1}) + alpha2 dt^2/2 R2(w_{l-1}).

Correct (Eq. corrector with Eq. nonlinear_corrector, alpha1 = alpha2 = 1):
for k = 0..k_max-1 and each l = 2..s, using iterate [k] of every stage,
    I_l = dt sum_j B1[l][j] R1(w_j^[k]) + dt^2 sum_j B2[l][j] R2(w_j^[k])
    W - dt R1(W) + dt^2/2 R2(W) = w_1 - dt R1(w_l^[k]) + dt^2/2 R2(w_l^[k]) + I_l
    -> w_l^[k+1] = W.
  (Eq. nonlinear_corrector prints b without I_l; the corrector equation it is
  derived from contains I_l, so b includes it.  The stage solves of one sweep
  are independent of each other.)

Update: w^{n+1} = w_s^[k_max] (first-same-as-last).

In the explicit terms R2(w) means R2(w, R1(w)).

The driver is generic: w may be a NumPy array or any object with +, - and
multiplication by a scalar (the tests use exact power series for the
Dahlquist problem).  `solve(b, a1dt, bcoef, guess)` must return W.
"""
from fractions import Fraction
from .tableaux import tableau


def hbpc_step(w, dt, q, kmax, R1, R2, solve, record=None):
    tab = tableau(q)
    s = tab.s
    exact = isinstance(dt, Fraction)          # exact rational arithmetic (symbolic tests)
    cv = (lambda x: x) if exact else float
    if not exact:
        dt = float(dt)
    c = [cv(x) for x in tab.c]
    B1 = [[cv(x) for x in row] for row in tab.B1]
    B2 = [[cv(x) for x in row] for row in tab.B2]

    W = [None] * s
    r1 = [None] * s
    r2 = [None] * s
    W[0] = w
    r1[0], r2[0] = R1(w), R2(w)

    # predictor
    for l in range(1, s):
        dc = c[l] - c[l - 1]
        a1dt = dc / 2 * dt
        bcoef = dc * dc / 6 * dt * dt / 2
        b = W[l - 1] + r1[l - 1] * a1dt + r2[l - 1] * bcoef
        W[l] = solve(b, a1dt, bcoef, W[l - 1])
        r1[l], r2[l] = R1(W[l]), R2(W[l])
        if record is not None:
            record.append(("predict", l))

    # corrector sweeps (Jacobi in l: all solves use iterate [k])
    for k in range(kmax):
        Wn = list(W)
        for l in range(1, s):
            I = None
            for j in range(s):
                t = r1[j] * (dt * B1[l][j]) + r2[j] * (dt * dt * B2[l][j])
                I = t if I is None else I + t
            b = W[0] - r1[l] * dt + r2[l] * (dt * dt / 2) + I
            Wn[l] = solve(b, dt, dt * dt / 2, W[l])
            if record is not None:
                record.append(("correct", k, l))
        W = Wn
        if k < kmax - 1:
            for l in range(1, s):
                r1[l], r2[l] = R1(W[l]), R2(W[l])
    return W[s - 1]
