"""An independent, high-precision evaluation of one Runge-Kutta stage on tiny grids.

Used only to pin the oracle.  It is built differently from the oracle on purpose:
  * ghost cells are explicit padded arrays, two layers deep, filled by mirroring across walls
    (rho, p kept, velocity negated: both components for no-slip, the normal one for free
    slip) or by periodic copies, corners receiving both fills
    (Sec. 2.5 and the oracle's reading of it), instead of per-face virtual stencils;
  * |A| comes from mpmath's eigendecomposition of the Jacobian printed in Sec. 2.1.3, not from
    the printed eigenvector matrices;
  * y-faces are handled by exchanging u and v (the rotation of Algorithm 2 for n = (0, 1));
  * arithmetic is mpmath at 40 significant digits.
Only plain boxes (no solid cells) are supported.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 40
WALL, PERIODIC = 0, 1


def G(a, b, k):
    s = 1 if b > 0 else (-1 if b < 0 else 0)
    return s * max(0, min(k * abs(b), s * a), min(abs(b), k * s * a))


def absA(q, beta):
    rho, u, v = q[0], q[1] / q[0], q[2] / q[0]
    A = mp.matrix([[0, 1, 0, 0],
                   [-u * u, 2 * u, 0, beta],
                   [-u * v, v, u, 0],
                   [-u / rho, 1 / rho, 0, 0]])
    # A + sigma I has the same eigenvectors; a shift helps mpmath's QR where it stalls
    for sigma in (0, mp.mpf("0.3713"), mp.mpf("-1.917"), mp.mpf("5.31")):
        try:
            E, V = mp.eig(A + sigma * mp.eye(4))
            break
        except RuntimeError:
            continue
    E = [e - sigma for e in E]
    Lam = mp.diag([abs(mp.re(e)) for e in E])
    M = V * Lam * mp.inverse(V)
    return mp.matrix([[mp.re(M[i, j]) for j in range(4)] for i in range(4)])


def phys(q, beta):
    u = q[1] / q[0]
    return [q[1], q[1] * u + beta * q[3], q[2] * u, u]


def osher(ql, qr, beta):
    xs = [-mp.sqrt(mp.mpf(3) / 5), mp.mpf(0), mp.sqrt(mp.mpf(3) / 5)]
    ws = [mp.mpf(5) / 9, mp.mpf(8) / 9, mp.mpf(5) / 9]
    dq = mp.matrix([qr[i] - ql[i] for i in range(4)])
    integ = mp.matrix([0, 0, 0, 0])
    for x, w in zip(xs, ws):
        t = (x + 1) / 2
        qj = [ql[i] + dq[i] * t for i in range(4)]
        integ += (w / 2) * (absA(qj, beta) * dq)
    fl, fr = phys(ql, beta), phys(qr, beta)
    return [(fl[i] + fr[i] - integ[i]) / 2 for i in range(4)]


def stage(nx, ny, lx, ly, gx, gy, beta, bc, qprev, q0, qn, dt, alpha, cfl, k, slip=False):
    """qprev, q0, qn: float64 [4, ny, nx] with the pressure itself.  Backward Euler, local dtau.
    Returns a dict with prim, grad (8 planes), fx, fy, resid and qout as float64 arrays."""
    mpf = mp.mpf
    dx, dy = mpf(lx) / nx, mpf(ly) / ny
    beta, gx, gy, dt, alpha, cfl, k = map(mpf, (beta, gx, gy, dt, alpha, cfl, k))
    P = 2
    NX, NY = nx + 2 * P, ny + 2 * P

    # padded primitive arrays W[j][i] = [rho, u, v, p]; D[j][i] = [Drho, Dru, Drv]; rho0; gsign
    W = [[None] * NX for _ in range(NY)]
    D = [[None] * NX for _ in range(NY)]
    R0 = [[None] * NX for _ in range(NY)]
    GS = [[1] * NX for _ in range(NY)]
    for j in range(ny):
        for i in range(nx):
            r = mpf(qprev[0, j, i])
            W[j + P][i + P] = [r, mpf(qprev[1, j, i]) / r, mpf(qprev[2, j, i]) / r,
                               beta * (mpf(qprev[3, j, i]) / beta)]
            D[j + P][i + P] = [(mpf(q0[c, j, i]) - mpf(qn[c, j, i])) / dt for c in range(3)]
            R0[j + P][i + P] = mpf(q0[0, j, i])

    def mir_x(w):
        return [w[0], -w[1], w[2] if slip else -w[2]] + list(w[3:])

    def mir_y(w):
        return [w[0], w[1] if slip else -w[1], -w[2]] + list(w[3:])

    def fill(arr, mx, my):
        # x sides first (rows of the interior), then y sides over the full padded width
        for j in range(P, P + ny):
            for d in (1, 2):
                if bc[0] == PERIODIC:
                    arr[j][P - d] = list(arr[j][P + nx - d])
                else:
                    arr[j][P - d] = mx(arr[j][P + d - 1])
                if bc[1] == PERIODIC:
                    arr[j][P + nx - 1 + d] = list(arr[j][P + d - 1])
                else:
                    arr[j][P + nx - 1 + d] = mx(arr[j][P + nx - d])
        for i in range(NX):
            for d in (1, 2):
                if bc[2] == PERIODIC:
                    arr[P - d][i] = list(arr[P + ny - d][i])
                else:
                    arr[P - d][i] = my(arr[P + d - 1][i])
                if bc[3] == PERIODIC:
                    arr[P + ny - 1 + d][i] = list(arr[P + d - 1][i])
                else:
                    arr[P + ny - 1 + d][i] = my(arr[P + ny - d][i])

    fill(W, mir_x, mir_y)
    fill(D, mir_x, mir_y)     # D = (D_rho, D_rho u, D_rho v) mirrors like (rho, u, v)
    R0w = [[[x] if x is not None else None for x in row] for row in R0]
    fill(R0w, list, list)
    # gravity sign: reversed in wall ghosts (non-corner ring cells are what matter)
    for j in range(NY):
        for i in range(NX):
            inside_x = P <= i < P + nx
            inside_y = P <= j < P + ny
            rev = False
            if not inside_x and bc[0] != PERIODIC:
                rev = not rev
            if not inside_y and bc[2] != PERIODIC:
                rev = not rev
            GS[j][i] = -1 if rev else 1

    grad = {}
    gp = {}
    for j in range(1, NY - 1):
        for i in range(1, NX - 1):
            c = W[j][i]
            if c is None or W[j][i - 1] is None or W[j][i + 1] is None or W[j - 1][i] is None \
                    or W[j + 1][i] is None:
                continue
            gxv = [G((W[j][i + 1][f] - c[f]) / dx, (c[f] - W[j][i - 1][f]) / dx, k) for f in range(3)]
            gyv = [G((W[j + 1][i][f] - c[f]) / dy, (c[f] - W[j - 1][i][f]) / dy, k) for f in range(3)]
            grad[(j, i)] = (gxv, gyv)
            r, u, v = c[0], c[1], c[2]
            rx, ux, vx = gxv
            ry, uy, vy = gyv
            Dc, rho0, sg = D[j][i], R0w[j][i][0], GS[j][i]
            px = -Dc[1] - (u * u * rx + 2 * r * u * ux) - (u * v * ry + r * u * vy + r * v * uy) + rho0 * gx * sg
            py = -Dc[2] - (u * v * rx + r * u * vx + r * v * ux) - (v * v * ry + 2 * r * v * vy) + rho0 * gy * sg
            gp[(j, i)] = (px, py)

    def state(j, i, di, dj):
        c = W[j][i]
        gxv, gyv = grad[(j, i)]
        px, py = gp[(j, i)]
        if di:
            h = dx / 2 * di
            r, u, v, p = c[0] + gxv[0] * h, c[1] + gxv[1] * h, c[2] + gxv[2] * h, c[3] + px * h
        else:
            h = dy / 2 * dj
            r, u, v, p = c[0] + gyv[0] * h, c[1] + gyv[1] * h, c[2] + gyv[2] * h, c[3] + py * h
        return [r, r * u, r * v, p / beta]

    fx = np.zeros((4, ny, nx + 1))
    fy = np.zeros((4, ny + 1, nx))
    FX, FY = {}, {}
    for j in range(ny):
        for f in range(nx + 1):
            jj, il, ir = j + P, f + P - 1, f + P
            F = osher(state(jj, il, +1, 0), state(jj, ir, -1, 0), beta)
            FX[(j, f)] = F
            fx[:, j, f] = [float(x) for x in F]
    sw = [0, 2, 1, 3]
    for f in range(ny + 1):
        for i in range(nx):
            ii, jl, jr = i + P, f + P - 1, f + P
            a, b = state(jl, ii, 0, +1), state(jr, ii, 0, -1)
            F = osher([a[m] for m in sw], [b[m] for m in sw], beta)
            F = [F[m] for m in sw]
            FY[(f, i)] = F
            fy[:, f, i] = [float(x) for x in F]

    prim = np.zeros((4, ny, nx))
    gout = np.zeros((8, ny, nx))
    resid = np.zeros((4, ny, nx))
    qout = np.zeros((4, ny, nx))
    dtau = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            jj, ii = j + P, i + P
            prim[:, j, i] = [float(x) for x in W[jj][ii]]
            gxv, gyv = grad[(jj, ii)]
            gout[:, j, i] = [float(x) for x in gxv] + [float(gp[(jj, ii)][0])] + \
                [float(x) for x in gyv] + [float(gp[(jj, ii)][1])]
            r0 = mpf(q0[0, j, i])
            u0, v0 = mpf(q0[1, j, i]) / r0, mpf(q0[2, j, i]) / r0
            cx = mp.sqrt(u0 * u0 + 4 * beta / r0)
            cy = mp.sqrt(v0 * v0 + 4 * beta / r0)
            dtau_c = cfl * dx * dy / ((abs(u0) + cx) / 2 * dy + (abs(v0) + cy) / 2 * dx)
            dtau[j, i] = float(dtau_c)
            body = [0, r0 * gx, r0 * gy, 0]
            Dk = list(D[jj][ii]) + [0]
            q0v = [mpf(q0[0, j, i]), mpf(q0[1, j, i]), mpf(q0[2, j, i]), mpf(q0[3, j, i]) / beta]
            for c in range(4):
                br = -((FX[(j, i + 1)][c] - FX[(j, i)][c]) / dx + (FY[(j + 1, i)][c] - FY[(j, i)][c]) / dy) \
                    - Dk[c] + body[c]
                api = 1 + alpha * dtau_c / dt if c < 3 else 1
                qn_c = q0v[c] + alpha * dtau_c / api * br
                resid[c, j, i] = float(br * beta if c == 3 else br)
                qout[c, j, i] = float(qn_c * beta if c == 3 else qn_c)
    return {"prim": prim, "grad": gout, "fx": fx, "fy": fy, "resid": resid, "qout": qout,
            "dtau": dtau}
