"""A second, independent implementation of one lattice Boltzmann step, written
as scalar loops over nodes in pure Python (float64), for tiny grids only.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

It deliberately shares nothing with the vectorised oracle modules: velocities,
weights, the Hermite rows, the inverse transform (closed form from the
weighted orthogonality of the Hermite basis instead of a linear solve), the
group elements and their action are all rebuilt here from the definitions in
Sec. II.A/II.B, in a different style, so that a slip in one implementation
shows up as a disagreement with the other.

Populations are nested lists f[i][z][y][x] or numpy arrays of that shape.
"""
import itertools
import math

SQ3 = math.sqrt(3.0)

VEL = [(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)]
W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
WEIGHT = [W1[a] * W1[b] * W1[c] for (a, b, c) in VEL]

# Multi-indices of the Hermite rows in the printed order of Sec. II.B.
ROWS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
        (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2),
        (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 2, 1), (0, 1, 2),
        (2, 2, 0), (2, 1, 1), (2, 0, 2), (1, 2, 1), (1, 1, 2), (0, 2, 2),
        (2, 2, 1), (2, 1, 2), (1, 2, 2),
        (2, 2, 2)]


def he(n, x):
    """He_0 = 1, He_1 = x, He_2 = x^2 - 1."""
    return 1.0 if n == 0 else (x if n == 1 else x * x - 1.0)


HROW = [[he(nx, SQ3 * c[0]) * he(ny, SQ3 * c[1]) * he(nz, SQ3 * c[2]) for c in VEL]
        for (nx, ny, nz) in ROWS]
# Weighted norms sum_i w_i H_k(xi_i)^2; the inverse follows from orthogonality:
# (M^{-1})_{ik} = w_i H_k(xi_i) / norm_k.
NORM = [sum(WEIGHT[i] * HROW[k][i] ** 2 for i in range(27)) for k in range(27)]
ORDER = [sum(r) for r in ROWS]


def group_elements():
    """O_h as functions acting on a velocity tuple."""
    out = []
    for perm in itertools.permutations((0, 1, 2)):
        for sg in itertools.product((1, -1), repeat=3):
            out.append((perm, sg))
    return out


def act(elem, c):
    perm, sg = elem
    return tuple(sg[r] * c[perm[r]] for r in range(3))


def feq_node(rho, u):
    out = []
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    for i, c in enumerate(VEL):
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        out.append(WEIGHT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu))
    return out


def phi(x, layers, act_name):
    h = list(x)
    for li, (W, b) in enumerate(layers):
        nxt = []
        for o in range(len(b)):
            s = b[o]
            for a in range(len(h)):
                s += h[a] * W[a][o]
            if li < len(layers) - 1:
                s = math.tanh(s) if act_name == "tanh" else max(s, 0.0)
            nxt.append(s)
        h = nxt
    return h


def collide_node(fn, kind, tau, omega_high=None, layers=None, act_name="tanh"):
    rho = sum(fn)
    u = [sum(VEL[i][a] * fn[i] for i in range(27)) / rho for a in range(3)]
    feq = feq_node(rho, u)
    if kind == "bgk":
        return [fn[i] - (fn[i] - feq[i]) / tau for i in range(27)]
    m = [sum(HROW[k][i] * fn[i] for i in range(27)) for k in range(27)]
    meq = [sum(HROW[k][i] * feq[i] for i in range(27)) for k in range(27)]
    if kind == "nco":
        index = {c: i for i, c in enumerate(VEL)}
        tt = [0.0] * 4
        elems = group_elements()
        for e in elems:
            fg = [0.0] * 27
            for j, c in enumerate(VEL):
                fg[index[act(e, c)]] = fn[j]
            mg = [sum(HROW[k][i] * fg[i] for i in range(27)) for k in range(27)]
            y = phi(mg, layers, act_name)
            tt = [tt[n] + y[n] / len(elems) for n in range(4)]
        omega_high = [1.0 / (0.5 + 0.5 / (1.0 + math.exp(t))) for t in tt]
    s = []
    for k in range(27):
        s.append(1.0 if ORDER[k] <= 1 else (1.0 / tau if ORDER[k] == 2 else omega_high[ORDER[k] - 3]))
    dm = [s[k] * (m[k] - meq[k]) for k in range(27)]
    return [fn[i] - sum(WEIGHT[i] * HROW[k][i] / NORM[k] * dm[k] for k in range(27))
            for i in range(27)]


def step(f, kind, tau, omega_high=None, layers=None, act_name="tanh"):
    """One pull-stream + collide step over a tiny periodic grid."""
    nz, ny, nx = len(f[0]), len(f[0][0]), len(f[0][0][0])
    out = [[[[0.0] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(27)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                fn = []
                for i, (cx, cy, cz) in enumerate(VEL):
                    fn.append(float(f[i][(z - cz) % nz][(y - cy) % ny][(x - cx) % nx]))
                post = collide_node(fn, kind, tau, omega_high, layers, act_name)
                for i in range(27):
                    out[i][z][y][x] = post[i]
    return out
