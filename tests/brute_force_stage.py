"""An independent, high-precision evaluation of one Runge-Kutta stage on tiny grids.

Used only to pin the oracle.  It is built differently from the oracle on purpose:
  * ghost cells are explicit padded arrays, two layers deep, filled by mirroring across walls
    (rho, p kept, velocity negated: both components for no-slip, the normal one for free
    slip) or by periodic copies, corners receiving both fills
    (Sec. 2.5 and the oracle's reading of it), instead of per-face virtual stencils;
  * |A| comes from mpmath's eigendecomposition of the Jacobian printed in Sec. 2.1.3, not from
    the printed eigenvector matrices;
  * y-faces are handled by exchanging u and v (the rotation of Algorithm 2 for n = (0, 1));
  * the exact (Bassi) flux solves the two p/beta jump conditions across the acoustic waves for
    u* and p* and the mass conditions for the star densities, instead of using the printed
    closed form;
  * arithmetic is mpmath at 40 significant digits.
Zero-gradient sides fill their ghosts like walls but without negating velocities or reversing
gravity.  Only plain boxes (no solid cells) are supported.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 40
WALL, PERIODIC, OPEN = 0, 1, 2


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


def roe(ql, qr, beta):
    rl, rr = ql[0], qr[0]
    sl, sr = mp.sqrt(rl), mp.sqrt(rr)
    ut = (sl * ql[1] / rl + sr * qr[1] / rr) / (sl + sr)
    vt = (sl * ql[2] / rl + sr * qr[2] / rr) / (sl + sr)
    rt = mp.sqrt(rl * rr)
    dq = mp.matrix([qr[i] - ql[i] for i in range(4)])
    d = absA([rt, rt * ut, rt * vt, 0], beta) * dq
    fl, fr = phys(ql, beta), phys(qr, beta)
    return [(fl[i] + fr[i] - d[i]) / 2 for i in range(4)]


def exact_state(ql, qr, beta, xi=0):
    rl, rr = ql[0], qr[0]
    ul, ur = ql[1] / rl, qr[1] / rr
    pl, pr = beta * ql[3], beta * qr[3]
    sl = (ul - mp.sqrt(ul * ul + 4 * beta / rl)) / 2
    sr = (ur + mp.sqrt(ur * ur + 4 * beta / rr)) / 2
    # u* - u_L = S_L (p* - p_L)/beta and u_R - u* = S_R (p_R - p*)/beta
    M = mp.matrix([[1, -sl / beta], [1, -sr / beta]])
    rhs = mp.matrix([ul - sl * pl / beta, ur - sr * pr / beta])
    us, ps = mp.lu_solve(M, rhs)
    if xi < sl:
        return list(ql)
    if xi < us:
        rs = rl * (ul - sl) / (us - sl)
        return [rs, rs * us, rs * ql[2] / rl, ps / beta]
    if xi < sr:
        rs = rr * (ur - sr) / (us - sr)
        return [rs, rs * us, rs * qr[2] / rr, ps / beta]
    return list(qr)


def bassi(ql, qr, beta):
    return phys(exact_state(ql, qr, beta), beta)


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


def stage(nx, ny, lx, ly, gx, gy, beta, bc, qprev, q0, qn, dt, alpha, cfl, k, slip=False,
          flux="osher", pgrad=0, pk=1, qnm1=None, qnm2=None, local=True):
    """qprev, q0, qn (qnm1, qnm2): float64 [4, ny, nx] with the pressure itself.  BDF order from
    the levels given; dt <= 0: no real-time term.  pgrad 0 new method, 1 k-limiter on p, 2 split
    limiter.  Returns a dict with prim, grad (8 planes), fx, fy, resid and qout as float64."""
    mpf = mp.mpf
    dx, dy = mpf(lx) / nx, mpf(ly) / ny
    pseudo_only = dt <= 0
    beta, gx, gy, dt, alpha, cfl, k, pk = map(mpf, (beta, gx, gy, dt, alpha, cfl, k, pk))
    B = [mpf(1), mpf(-1)]
    if qnm1 is not None and qnm2 is not None:
        B = [mpf(11) / 6, mpf(-3), mpf(3) / 2, mpf(-1) / 3]
    elif qnm1 is not None:
        B = [mpf(3) / 2, mpf(-2), mpf(1) / 2]
    levels = [q0, qn, qnm1, qnm2][:len(B)]
    riemann = {"osher": osher, "roe": roe, "bassi": bassi}[flux]
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
            D[j + P][i + P] = [0 if pseudo_only else
                               sum(b * mpf(lv[c, j, i]) for b, lv in zip(B, levels)) / dt
                               for c in range(3)]
            R0[j + P][i + P] = mpf(q0[0, j, i])

    def mir_x(w):
        return [w[0], -w[1], w[2] if slip else -w[2]] + list(w[3:])

    def mir_y(w):
        return [w[0], w[1] if slip else -w[1], -w[2]] + list(w[3:])

    def fill(arr, mx, my):
        # x sides first (rows of the interior), then y sides over the full padded width; a
        # zero-gradient side copies the mirror position unchanged
        def img(side, w, m):
            return list(w) if bc[side] == OPEN else m(w)
        for j in range(P, P + ny):
            for d in (1, 2):
                if bc[0] == PERIODIC:
                    arr[j][P - d] = list(arr[j][P + nx - d])
                else:
                    arr[j][P - d] = img(0, arr[j][P + d - 1], mx)
                if bc[1] == PERIODIC:
                    arr[j][P + nx - 1 + d] = list(arr[j][P + d - 1])
                else:
                    arr[j][P + nx - 1 + d] = img(1, arr[j][P + nx - d], mx)
        for i in range(NX):
            for d in (1, 2):
                if bc[2] == PERIODIC:
                    arr[P - d][i] = list(arr[P + ny - d][i])
                else:
                    arr[P - d][i] = img(2, arr[P + d - 1][i], my)
                if bc[3] == PERIODIC:
                    arr[P + ny - 1 + d][i] = list(arr[P + d - 1][i])
                else:
                    arr[P + ny - 1 + d][i] = img(3, arr[P + ny - d][i], my)

    fill(W, mir_x, mir_y)
    fill(D, mir_x, mir_y)     # D = (D_rho, D_rho u, D_rho v) mirrors like (rho, u, v)
    R0w = [[[x] if x is not None else None for x in row] for row in R0]
    fill(R0w, list, list)
    # gravity sign: reversed in wall ghosts (non-corner ring cells are what matter)
    for j in range(NY):
        for i in range(NX):
            rev = False
            if i < P and bc[0] == WALL or i >= P + nx and bc[1] == WALL:
                rev = not rev
            if j < P and bc[2] == WALL or j >= P + ny and bc[3] == WALL:
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
            if pgrad == 1:
                px = G((W[j][i + 1][3] - c[3]) / dx, (c[3] - W[j][i - 1][3]) / dx, pk)
                py = G((W[j + 1][i][3] - c[3]) / dy, (c[3] - W[j - 1][i][3]) / dy, pk)
            elif pgrad == 2:
                gxs, gys = gx * sg, gy * sg
                kxr = (W[j][i + 1][3] - c[3]) / dx - (c[0] + W[j][i + 1][0]) * gxs / 2
                kxl = (c[3] - W[j][i - 1][3]) / dx - (W[j][i - 1][0] + c[0]) * gxs / 2
                kyr = (W[j + 1][i][3] - c[3]) / dy - (c[0] + W[j + 1][i][0]) * gys / 2
                kyl = (c[3] - W[j - 1][i][3]) / dy - (W[j - 1][i][0] + c[0]) * gys / 2
                px = c[0] * gxs + G(kxr, kxl, pk)
                py = c[0] * gys + G(kyr, kyl, pk)
            else:
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
            F = riemann(state(jj, il, +1, 0), state(jj, ir, -1, 0), beta)
            FX[(j, f)] = F
            fx[:, j, f] = [float(x) for x in F]
    sw = [0, 2, 1, 3]
    for f in range(ny + 1):
        for i in range(nx):
            ii, jl, jr = i + P, f + P - 1, f + P
            a, b = state(jl, ii, 0, +1), state(jr, ii, 0, -1)
            F = riemann([a[m] for m in sw], [b[m] for m in sw], beta)
            F = [F[m] for m in sw]
            FY[(f, i)] = F
            fy[:, f, i] = [float(x) for x in F]

    prim = np.zeros((4, ny, nx))
    gout = np.zeros((8, ny, nx))
    resid = np.zeros((4, ny, nx))
    qout = np.zeros((4, ny, nx))
    dtau = np.zeros((ny, nx))
    dtau_mp = {}
    for j in range(ny):
        for i in range(nx):
            r0 = mpf(q0[0, j, i])
            u0, v0 = mpf(q0[1, j, i]) / r0, mpf(q0[2, j, i]) / r0
            cx = mp.sqrt(u0 * u0 + 4 * beta / r0)
            cy = mp.sqrt(v0 * v0 + 4 * beta / r0)
            dtau_mp[(j, i)] = cfl * dx * dy / ((abs(u0) + cx) / 2 * dy + (abs(v0) + cy) / 2 * dx)
    if not local:
        m = min(dtau_mp.values())
        dtau_mp = {key: m for key in dtau_mp}
    for j in range(ny):
        for i in range(nx):
            jj, ii = j + P, i + P
            prim[:, j, i] = [float(x) for x in W[jj][ii]]
            gxv, gyv = grad[(jj, ii)]
            gout[:, j, i] = [float(x) for x in gxv] + [float(gp[(jj, ii)][0])] + \
                [float(x) for x in gyv] + [float(gp[(jj, ii)][1])]
            r0 = mpf(q0[0, j, i])
            dtau_c = dtau_mp[(j, i)]
            dtau[j, i] = float(dtau_c)
            body = [0, r0 * gx, r0 * gy, 0]
            Dk = list(D[jj][ii]) + [0]
            q0v = [mpf(q0[0, j, i]), mpf(q0[1, j, i]), mpf(q0[2, j, i]), mpf(q0[3, j, i]) / beta]
            for c in range(4):
                br = -((FX[(j, i + 1)][c] - FX[(j, i)][c]) / dx + (FY[(j + 1, i)][c] - FY[(j, i)][c]) / dy) \
                    - Dk[c] + body[c]
                api = 1 + B[0] * alpha * dtau_c / dt if c < 3 and not pseudo_only else 1
                qn_c = q0v[c] + alpha * dtau_c / api * br
                resid[c, j, i] = float(br * beta if c == 3 else br)
                qout[c, j, i] = float(qn_c * beta if c == 3 else qn_c)
    return {"prim": prim, "grad": gout, "fx": fx, "fy": fy, "resid": resid, "qout": qout,
            "dtau": dtau}
