"""Brute-force transcription of the penalized LBM step for tiny lattices.

TEST INFRASTRUCTURE ONLY.  Pure Python over dicts of nodes, written apart from
the C oracle (different layout, push-style streaming, whole-lattice indicator
scan, explicit tensors) so that the two cross-check each other.  Each function
cites the passage of Millet & Liberge (arXiv 2511.01629) it restates.
"""
import math

CS2 = 1.0 / 3.0


def velocities(kind):
    """D2Q9 in the numbering of the velocity-set figure (sec. 2.2); D3Q19 with
    rest, the six faces, then the twelve edges (opposites adjacent)."""
    if kind == "D2Q9":
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
             (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
        wt = {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}
    else:
        c = [(0, 0, 0)]
        for k in range(3):
            for s in (1, -1):
                v = [0, 0, 0]
                v[k] = s
                c.append(tuple(v))
        for (i, j) in ((0, 1), (0, 2), (1, 2)):
            for (si, sj) in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
                v = [0, 0, 0]
                v[i], v[j] = si, sj
                c.append(tuple(v))
        wt = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    w = [wt[sum(x * x for x in v)] for v in c]
    return c, w


def dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def feq(c, w, p, u):
    """sec. 2.2 eq. (13)"""
    uu = dot(u, u)
    out = []
    for a, ca in enumerate(c):
        if a == 0:
            out.append(-(1 - w[0]) * p / CS2 - w[0] * uu / (2 * CS2))
        else:
            cu = dot(ca, u)
            out.append(w[a] * (p / CS2 + cu / CS2 + cu * cu / (2 * CS2 ** 2) - uu / (2 * CS2)))
    return out


def step(state):
    """One step n -> n+1 on a state dict; returns a new state dict.

    state = dict(kind, n=(nx,ny,nz), periodic=(..), tau, alpha, rho_f, g,
                 eps_p, eps_w, delta, K, f={node: [Q floats]},
                 parts=[dict(shape, rho_s, a, b, X, theta, Uprev, Wprev, A)])
    """
    kind = state["kind"]
    c, w = velocities(kind)
    Q = len(c)
    d = 2 if kind == "D2Q9" else 3
    nx, ny, nz = state["n"]
    per = state["periodic"]
    tau, alpha = state["tau"], state["alpha"]
    parts = state["parts"]
    nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]

    # S1: whole-lattice scan, lowest id wins (sec. 2.1 eq. 9)
    def disp(node, X):
        r = []
        for k in range(d):
            t = node[k]
            if per[k]:
                if t - X[k] > state["n"][k] / 2:
                    t -= state["n"][k]
                elif t - X[k] < -state["n"][k] / 2:
                    t += state["n"][k]
            r.append(float(t) - X[k])
        while len(r) < 3:
            r.append(0.0)
        return r

    def inside(pt, r):
        if pt["shape"] == "disk":
            return r[0] * r[0] + r[1] * r[1] <= pt["a"] * pt["a"]
        if pt["shape"] == "sphere":
            return r[0] * r[0] + r[1] * r[1] + r[2] * r[2] <= pt["a"] * pt["a"]
        cs, sn = math.cos(pt["theta"]), math.sin(pt["theta"])
        xi = cs * r[0] + sn * r[1]
        eta = -sn * r[0] + cs * r[1]
        a, b = pt["a"], pt["b"]
        return (b * b) * (xi * xi) + (a * a) * (eta * eta) <= (a * a) * (b * b)

    # the fractional indicator (an extension, disks and spheres): the band
    # |r| < R + 1/2 with chi = min(1, R + 1/2 - |r|), the first particle whose
    # band holds the node owns it; chi = 1 on the nodes of the binary indicator
    frac = state.get("fractional", False)
    owner, chi = {}, {}
    for nd in nodes:
        owner[nd], chi[nd] = -1, 0.0
        for i, pt in enumerate(parts):
            r = disp(nd, pt["X"])
            if frac:
                r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2]
                if r2 < (pt["a"] + 0.5) * (pt["a"] + 0.5):
                    owner[nd], chi[nd] = i, min(1.0, pt["a"] + 0.5 - math.sqrt(r2))
                    break
            elif inside(pt, r):
                owner[nd], chi[nd] = i, 1.0
                break

    # S2/S3: acceleration and macroscopic fields (eq. 15a-b)
    def accel(nd):
        i = owner[nd]
        if i < 0:
            return [0.0, 0.0, 0.0]
        pt = parts[i]
        b = 1.0 - state["rho_f"] / pt["rho_s"]
        return [chi[nd] * (b * state["g"][k] + pt["A"][k]) if k < d else 0.0 for k in range(3)]

    f = state["f"]
    U, P = {}, {}
    for nd in nodes:
        acc = accel(nd)
        fv = f[nd]
        u = [sum(fv[a] * c[a][k] for a in range(Q)) + acc[k] / 2 for k in range(3)]
        p = (CS2 * sum(fv[1:]) - w[0] / 2 * dot(u, u)) / (1 - w[0])
        U[nd], P[nd] = u, p

    # S4: discrete momentum sums (sec. 2.4, eq. 22a-b)
    meas = []
    for i, pt in enumerate(parts):
        own = [nd for nd in nodes if owner[nd] == i]
        N = sum(chi[nd] for nd in own)  # the node count, or sum chi
        su = [sum(chi[nd] * U[nd][k] for nd in own) for k in range(3)]
        Uv = [s / N for s in su]
        rs = [disp(nd, pt["X"]) for nd in own]
        if d == 2:
            L = sum(chi[nd] * (r[0] * U[nd][1] - r[1] * U[nd][0]) for r, nd in zip(rs, own))
            I2 = sum(chi[nd] * (r[0] * r[0] + r[1] * r[1]) for r, nd in zip(rs, own))
            W = [0.0, 0.0, L / I2]
        else:
            Lv = [0.0, 0.0, 0.0]
            T = [[0.0] * 3 for _ in range(3)]
            for r, nd in zip(rs, own):
                u = U[nd]
                cr = [r[1] * u[2] - r[2] * u[1], r[2] * u[0] - r[0] * u[2], r[0] * u[1] - r[1] * u[0]]
                for k in range(3):
                    Lv[k] += chi[nd] * cr[k]
                rr = dot(r, r)
                for a in range(3):
                    for b in range(3):
                        T[a][b] += chi[nd] * ((rr if a == b else 0.0) - r[a] * r[b])
            W = solve3(T, Lv)
        meas.append((N, Uv, W))

    # S5: collision (eq. 10, 13, 14, 17); with the rigid-velocity forcing (an
    # extension, beta > 0) a solid node's acceleration gains
    # 2 beta (U_i + omega_i x r - u), u the fluid velocity of S3
    beta = state.get("beta", 0.0)
    stress = not state.get("no_stress_penalty", False)
    post = {}
    for nd in nodes:
        i = owner[nd]
        acc = accel(nd)
        u, p, fv = U[nd], P[nd], f[nd]
        if i >= 0 and beta > 0:
            _, Ui, Wi = meas[i]
            r = disp(nd, parts[i]["X"])
            rigid = [Ui[0] + Wi[1] * r[2] - Wi[2] * r[1], Ui[1] + Wi[2] * r[0] - Wi[0] * r[2],
                     Ui[2] + Wi[0] * r[1] - Wi[1] * r[0]]
            acc = [acc[k] + (2 * beta * (rigid[k] - u[k]) if k < d else 0.0) for k in range(3)]
            u = [sum(fv[a] * c[a][k] for a in range(Q)) + acc[k] / 2 for k in range(3)]
            p = (CS2 * sum(fv[1:]) - w[0] / 2 * dot(u, u)) / (1 - w[0])
        fe = feq(c, w, p, u)
        Pi = [[sum((fv[a] - fe[a]) * c[a][r] * c[a][s] for a in range(Q)) for s in range(3)] for r in range(3)]
        trPi = sum(Pi[k][k] for k in range(d))
        out = []
        for a in range(Q):
            ca = c[a]
            cu = dot(ca, u)
            F = (1 - 1 / (2 * tau)) * w[a] * sum(((ca[k] - u[k]) / CS2 + cu * ca[k] / CS2 ** 2) * acc[k] for k in range(3))
            S = 0.0
            if i >= 0 and stress:
                PiCC = sum(Pi[r][s] * ca[r] * ca[s] for r in range(3) for s in range(3))
                S = w[a] / (2 * CS2 ** 2) * alpha * chi[nd] * (PiCC - CS2 * trPi)
            out.append(fv[a] - (fv[a] - fe[a]) / tau + F + S)
        post[nd] = out

    # S6: push streaming; a population leaving through a wall returns reversed
    opp = [c.index(tuple(-x for x in v)) for v in c]
    newf = {nd: [None] * Q for nd in nodes}
    for nd in nodes:
        for a in range(Q):
            dst = list(nd)
            hit = False
            for k in range(3):
                dst[k] += c[a][k]
                if dst[k] < 0 or dst[k] >= state["n"][k]:
                    if per[k]:
                        dst[k] %= state["n"][k]
                    else:
                        hit = True
            if hit:
                newf[nd][opp[a]] = post[nd][a]
            else:
                newf[tuple(dst)][a] = post[nd][a]

    # S7: Algorithm 1 (sec. 2.4) with the collision forces of sec. 2.3
    K = state["K"]
    gmag = math.sqrt(dot(state["g"], state["g"]))

    def Cc(pt):
        V = {"disk": math.pi * pt["a"] ** 2, "ellipse": math.pi * pt["a"] * pt["b"],
             "sphere": 4.0 / 3.0 * math.pi * pt["a"] ** 3}[pt["shape"]]
        return (pt["rho_s"] - state["rho_f"]) * gmag * V

    def force(i, Y):
        pt = parts[i]
        F = [0.0, 0.0, 0.0]
        Ri, dl = pt["a"], state["delta"]
        for j, q in enumerate(parts):
            if j == i:
                continue
            dv = [Y[i][k] - Y[j][k] for k in range(3)]
            for k in range(d):
                if per[k]:
                    if dv[k] > state["n"][k] / 2:
                        dv[k] -= state["n"][k]
                    elif dv[k] < -state["n"][k] / 2:
                        dv[k] += state["n"][k]
            dist = math.sqrt(dot(dv, dv))
            if dist <= Ri + q["a"] + dl:
                m = Cc(pt) / state["eps_p"] * ((Ri + q["a"] + dl - dist) / dl) ** 2
                for k in range(3):
                    F[k] += m * dv[k] / dist
        for k in range(d):
            if per[k]:
                continue
            for wall in (-0.5, state["n"][k] - 0.5):
                mirror = 2 * wall - Y[i][k]
                dd = abs(Y[i][k] - mirror)
                if dd <= 2 * Ri + dl:
                    m = Cc(pt) / state["eps_w"] * ((2 * Ri + dl - dd) / dl) ** 2
                    F[k] += m * (Y[i][k] - mirror) / dd
        return F

    Ub = [[(meas[i][1][k] + pt["Uprev"][k]) / 2 for k in range(3)] for i, pt in enumerate(parts)]
    Y = [list(pt["X"]) for pt in parts]
    # X^{n+1} - X^n - U_bar is the sum of the correction displacements
    disp = [[0.0, 0.0, 0.0] for _ in parts]
    for _ in range(K):
        Ys = [[Y[i][k] + (Ub[i][k] / K if k < d else 0.0) for k in range(3)] for i in range(len(parts))]
        F0 = [force(i, Y) for i in range(len(parts))]
        F1 = [force(i, Ys) for i in range(len(parts))]
        corr = [[1 / (2 * parts[i]["rho_s"] * meas[i][0]) / K ** 2 * (F0[i][k] + F1[i][k]) / 2 if k < d else 0.0
                 for k in range(3)] for i in range(len(parts))]
        Y = [[Ys[i][k] + corr[i][k] for k in range(3)] for i in range(len(parts))]
        disp = [[disp[i][k] + corr[i][k] for k in range(3)] for i in range(len(parts))]
    newparts = []
    for i, pt in enumerate(parts):
        q = dict(pt)
        X = list(Y[i])
        q["A"] = [2 * disp[i][k] for k in range(3)]
        for k in range(d):
            if per[k]:
                if X[k] >= state["n"][k]:
                    X[k] -= state["n"][k]
                elif X[k] < 0:
                    X[k] += state["n"][k]
        q["X"] = X
        if d == 2:
            q["theta"] = pt["theta"] + (meas[i][2][2] + pt["Wprev"][2]) / 2
        q["Uprev"] = list(meas[i][1])
        q["Wprev"] = list(meas[i][2])
        q["N"] = meas[i][0]
        newparts.append(q)
    new = dict(state)
    new["f"] = newf
    new["parts"] = newparts
    new["owner"] = owner
    new["u"] = U
    return new


def solve3(T, b):
    def det(M):
        return (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]))
    D = det(T)
    out = []
    for col in range(3):
        M = [[b[r] if s == col else T[r][s] for s in range(3)] for r in range(3)]
        out.append(det(M) / D)
    return out


def initial_state(kind, n, periodic, tau, alpha, rho_f, g, u0, parts, eps_p=2.0, eps_w=1.0, delta=1.0, K=1,
                  beta=0.0, no_stress_penalty=False, fractional=False):
    """f = f^eq(0, u0) everywhere; U^{-1} = U^0 from the initial indicator."""
    c, w = velocities(kind)
    u0 = list(u0) + [0.0] * (3 - len(u0))
    g = list(g) + [0.0] * (3 - len(g))
    fe = feq(c, w, 0.0, u0)
    nodes = [(x, y, z) for z in range(n[2]) for y in range(n[1]) for x in range(n[0])]
    st = dict(kind=kind, n=tuple(n), periodic=tuple(periodic), tau=tau, alpha=alpha if alpha > 0 else 1.0 / tau,
              rho_f=rho_f, g=g, eps_p=eps_p, eps_w=eps_w, delta=delta, K=K, beta=beta,
              no_stress_penalty=no_stress_penalty, fractional=fractional,
              f={nd: list(fe) for nd in nodes}, parts=[])
    for pt in parts:
        q = dict(pt)
        q["X"] = list(pt["x"]) + [0.0] * (3 - len(pt["x"]))
        q.setdefault("b", pt["a"])
        q.setdefault("theta", 0.0)
        q["A"] = [0.0, 0.0, 0.0]
        q["Uprev"] = [0.0, 0.0, 0.0]
        q["Wprev"] = [0.0, 0.0, 0.0]
        st["parts"].append(q)
    # U^0 and omega^0: one dry evaluation of S1-S4 with zero collision force
    probe = step(dict(st, K=1, eps_p=1e300, eps_w=1e300))
    for q, qn in zip(st["parts"], probe["parts"]):
        q["Uprev"] = list(qn["Uprev"])
        q["Wprev"] = list(qn["Wprev"])
    return st
