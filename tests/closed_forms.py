"""Closed forms used as pins (independent of the oracle's stage recurrence)."""
import mpmath


def rk4_linear_closed_form(st, dt, nsteps, x0, v0, U):
    """Classical RK4 applied to the linear system y' = A y + b reduces to
    y_{n+1} = P4(dt A) y_n + dt Q3(dt A) b with P4(Z) = sum_{k<=4} Z^k/k! and
    Q3(Z) = sum_{k<=3} Z^k/(k+1)! (the stability polynomial form).  Here
    y = (x, v), A = [[0, 1], [0, -1/St]], b = (0, U/St): Stokes drag in a
    uniform flow.  Evaluated in 40-digit arithmetic."""
    mpmath.mp.dps = 40
    st, dt = mpmath.mpf(st), mpmath.mpf(dt)
    A = mpmath.matrix([[0, 1], [0, -1 / st]])
    b = mpmath.matrix([0, mpmath.mpf(U) / st])
    Z = dt * A
    I = mpmath.eye(2)
    P, Q, Zk = I * 0, I * 0, I
    for k in range(5):
        P += Zk / mpmath.factorial(k)
        if k <= 3:
            Q += Zk / mpmath.factorial(k + 1)
        Zk = Zk * Z
    c = dt * (Q * b)
    y = mpmath.matrix([mpmath.mpf(x0), mpmath.mpf(v0)])
    for _ in range(nsteps):
        y = P * y + c
    return float(y[0]), float(y[1])
