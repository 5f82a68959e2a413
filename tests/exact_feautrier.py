"""Exact rational solve of the discrete second-order Feautrier system: a checker
for the oracle, written independently of it (dense matrix, exact Gaussian
elimination)."""
from fractions import Fraction


def exact_u(dtau, S, m, I):
    """Solve the discrete system by exact rational Gaussian elimination.

    Rows: interior -A u_{d-1} + (1+A+C) u_d - C u_{d+1} = S_d with
    A = 2/(a(a+b)), C = 2/(b(a+b)), a = dtau_{d-1}, b = dtau_d; boundary
    rows from u' = u - I (second order): (1 + 2/h + 2/h^2) u_0 - 2/h^2 u_1 =
    S_0 + 2 I/h, mirrored at the far end.  Built as a dense matrix."""
    N = len(S)
    Fr = Fraction
    dt = [x if isinstance(x, Fr) else Fr(float(x)) for x in dtau]
    s = [x if isinstance(x, Fr) else Fr(float(x)) for x in S]
    I = I if isinstance(I, Fr) else Fr(float(I))
    if N == 1:
        return I
    M = [[Fr(0)] * N for _ in range(N)]
    rhs = [Fr(0)] * N
    h = dt[0]
    M[0][0] = 1 + 2 / h + 2 / (h * h)
    M[0][1] = -2 / (h * h)
    rhs[0] = s[0] + 2 * I / h
    h = dt[N - 2]
    M[N - 1][N - 1] = 1 + 2 / h + 2 / (h * h)
    M[N - 1][N - 2] = -2 / (h * h)
    rhs[N - 1] = s[N - 1] + 2 * I / h
    for d in range(1, N - 1):
        a, b = dt[d - 1], dt[d]
        A = 2 / (a * (a + b))
        C = 2 / (b * (a + b))
        M[d][d - 1] = -A
        M[d][d] = 1 + A + C
        M[d][d + 1] = -C
        rhs[d] = s[d]
    for c in range(N):  # Gaussian elimination, exact
        piv = next(r for r in range(c, N) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        rhs[c], rhs[piv] = rhs[piv], rhs[c]
        for r in range(c + 1, N):
            if M[r][c] != 0:
                f = M[r][c] / M[c][c]
                for k in range(c, N):
                    M[r][k] -= f * M[c][k]
                rhs[r] -= f * rhs[c]
    u = [Fr(0)] * N
    for c in range(N - 1, -1, -1):
        u[c] = (rhs[c] - sum(M[c][k] * u[k] for k in range(c + 1, N))) / M[c][c]
    return u[m]


def exact_u_tridiag(dtau, S, m, I):
    """The same system as exact_u, solved exactly by forward elimination and back
    substitution on its three diagonals (no pivoting is needed: the matrix is
    strictly diagonally dominant), so long refined lines stay cheap."""
    N = len(S)
    Fr = Fraction
    dt = [x if isinstance(x, Fr) else Fr(float(x)) for x in dtau]
    s = [x if isinstance(x, Fr) else Fr(float(x)) for x in S]
    I = I if isinstance(I, Fr) else Fr(float(I))
    if N == 1:
        return I
    lo, di, up, rhs = [Fr(0)] * N, [Fr(0)] * N, [Fr(0)] * N, [Fr(0)] * N
    h = dt[0]
    di[0], up[0], rhs[0] = 1 + 2 / h + 2 / (h * h), -2 / (h * h), s[0] + 2 * I / h
    h = dt[N - 2]
    di[N - 1], lo[N - 1], rhs[N - 1] = 1 + 2 / h + 2 / (h * h), -2 / (h * h), s[N - 1] + 2 * I / h
    for d in range(1, N - 1):
        a, b = dt[d - 1], dt[d]
        A, C = 2 / (a * (a + b)), 2 / (b * (a + b))
        lo[d], di[d], up[d], rhs[d] = -A, 1 + A + C, -C, s[d]
    for d in range(1, N):
        f = lo[d] / di[d - 1]
        di[d] -= f * up[d - 1]
        rhs[d] -= f * rhs[d - 1]
    u = [Fr(0)] * N
    u[N - 1] = rhs[N - 1] / di[N - 1]
    for d in range(N - 2, -1, -1):
        u[d] = (rhs[d] - up[d] * u[d + 1]) / di[d]
    return u[m]
