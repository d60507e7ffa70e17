"""Seeded synthetic lattice systems (no lattice-summation arithmetic here).

Seeds: numpy.random.default_rng(140500 + index) for the named workloads.

Named workloads
  1  box, b=10, n=64, L=2 (N=128): one unit charge at the centre of each of the
     8 lattice cells (a grid node), uniform sinc rule, M=20 (R=41). Full 128^3
     potential and the energy against a rank-8 density.
  2  box, b=10, n=128, L=32 (N=4096): 8 charges per cell on a rock-salt pattern
     shifted by 1/4 (+1 on one sublattice, -1 on the other) with a uniform
     jitter of at most 0.05 per fractional coordinate; rule S, M=47 (R=48);
     16 random 256^3 sub-boxes; rank-8 density.
  3  periodic, b=10, n=256, L=64 images per axis: 64 charges at uniform random
     positions, charges from {-2,-1,+1,+2} made neutral; rule S, M=59 (R=60).
  4  512 independent box systems: L in 4..48, n in {64,96,128,192,256}, M0 in
     1..32, uniform random positions, +-1 charges alternating then shuffled,
     R in {30,36,...,60}; per system the central unit cell is reconstructed.
  5  box, b=10, n=128, L=32: 64 charges at uniform random positions, 32 of
     each sign; rule S, M=47; forces.

Densities: rho(x) = sum_s d_s prod_l exp(-(x_l - c_{s,l})^2 / (2 sigma_s^2)),
d_s ~ U[0.5, 1.5], c_s uniform in the summation domain, sigma_s ~
U[0.05, 0.25] * (domain edge), sampled at cell midpoints (rank 8).
"""
import json
import os
from dataclasses import dataclass, field

import numpy as np

_TABLE = None


def _table():
    global _TABLE
    if _TABLE is None:
        with open(os.path.join(os.path.dirname(__file__), "rule_s.json")) as f:
            _TABLE = json.load(f)["table"]
    return _TABLE


def rule_s_params(M, X):
    """(C0, s_grid) of rule S for M and a master half-width of X cells: the
    tabulated entry with the same M and the smallest tabulated X >= X."""
    rows = [r for r in _table() if r["M"] == M and r["X"] >= X]
    if not rows:
        raise KeyError(f"no rule-S calibration for M={M}, X={X}")
    r = min(rows, key=lambda r: r["X"])
    return r["C0"], r["s"]


@dataclass
class Density:
    D: list          # three arrays (R_rho, N_l): factors sampled at cell midpoints
    d: np.ndarray    # (R_rho,) weights


@dataclass
class System:
    name: str
    b: float
    n: int
    L: tuple
    periodic: bool
    pos: np.ndarray          # (M0, 3) physical coordinates in [-b/2, b/2)
    Z: np.ndarray            # (M0,) charges
    quad: dict               # {"rule": "U"|"S", "M", "C0", "s"} (s in 1/length)
    density: Density = None
    boxes: np.ndarray = None  # (nbox, 6) int: origin(3), extent(3), in cells
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def h(self):
        return self.b / self.n

    @property
    def M0(self):
        return int(self.pos.shape[0])

    def N(self, l):
        return self.n if self.periodic else self.L[l] * self.n

    @property
    def R(self):
        return 2 * self.quad["M"] + 1 if self.quad["rule"] == "U" else self.quad["M"] + 1

    @property
    def K(self):
        return self.M0 * self.R


def _master_half_width(n, L, periodic):
    # cells from a charge to the far end of the summation domain, in cells
    if periodic:
        return max((Ll // 2 + 1) * n for Ll in L)
    return max(Ll * n for Ll in L)


def quad_spec(rule, M, n, L, periodic, b, C0=1.0):
    if rule == "U":
        return {"rule": "U", "M": int(M), "C0": float(C0), "s": 1.0}
    C0s, s_grid = rule_s_params(M, _master_half_width(n, L, periodic))
    return {"rule": "S", "M": int(M), "C0": float(C0s), "s": float(s_grid * n / b)}


def make_density(b, n, L, periodic, rng, R_rho=8, N=None):
    D = []
    if N is None:
        N = [n if periodic else L[l] * n for l in range(3)]
    lo = -0.5 * b
    edge = [N[l] * b / n for l in range(3)]
    d = rng.uniform(0.5, 1.5, R_rho)
    sig = rng.uniform(0.05, 0.25, R_rho) * float(np.mean(edge))
    centres = np.stack([rng.uniform(lo, lo + edge[l], R_rho) for l in range(3)], 1)
    for l in range(3):
        mid = lo + (np.arange(N[l]) + 0.5) * (b / n)
        D.append(np.exp(-((mid[None, :] - centres[:, l, None]) ** 2) / (2.0 * sig[:, None] ** 2)))
    return Density(D=D, d=d)


def frac_to_pos(frac, b):
    pos = -0.5 * b + np.asarray(frac, np.float64) * b
    return np.minimum(pos, np.nextafter(0.5 * b, 0.0))


def neutralise(Z, rng, levels=(-2, -1, 1, 2)):
    """Step charges toward neutrality inside the ordered set ``levels``
    (one unit where possible, +-1 -> -+1 otherwise), picking seeded atoms."""
    Z = np.array(Z, np.int64)
    lv = list(levels)
    while Z.sum() != 0:
        s = 1 if Z.sum() > 0 else -1
        # moves that change the total by exactly -s
        idx = [i for i in range(len(Z)) if Z[i] - s in lv and abs(Z[i] - s) > 0 and
               (Z[i] - s) * Z[i] > 0]
        if idx:
            i = idx[rng.integers(len(idx))]
            Z[i] -= s
            continue
        idx = [i for i in range(len(Z)) if Z[i] == s]
        i = idx[rng.integers(len(idx))]
        Z[i] = -s
    return Z.astype(np.float64)


def config1():
    rng = np.random.default_rng(140500 + 1)
    b, n, L = 10.0, 64, (2, 2, 2)
    pos = frac_to_pos([[0.5, 0.5, 0.5]], b)
    quad = quad_spec("U", 20, n, L, False, b, C0=1.0)
    dens = make_density(b, n, L, False, rng)
    boxes = np.array([[0, 0, 0, 128, 128, 128]], np.int64)
    return System("cfg1", b, n, L, False, pos, np.array([1.0]), quad, dens, boxes, 140501)


def config2():
    rng = np.random.default_rng(140500 + 2)
    b, n, L = 10.0, 128, (32, 32, 32)
    A = [(.25, .25, .25), (.25, .75, .75), (.75, .25, .75), (.75, .75, .25)]
    B = [(.75, .75, .75), (.75, .25, .25), (.25, .75, .25), (.25, .25, .75)]
    frac = np.array(A + B) + rng.uniform(-0.05, 0.05, (8, 3))
    Z = np.array([1.0] * 4 + [-1.0] * 4)
    quad = quad_spec("S", 47, n, L, False, b)
    dens = make_density(b, n, L, False, rng)
    N = L[0] * n
    org = rng.integers(0, N - 256 + 1, size=(16, 3))
    boxes = np.concatenate([org, np.full((16, 3), 256)], 1).astype(np.int64)
    return System("cfg2", b, n, L, False, frac_to_pos(frac, b), Z, quad, dens, boxes, 140502)


def config3():
    rng = np.random.default_rng(140500 + 3)
    b, n, L = 10.0, 256, (64, 64, 64)
    frac = rng.uniform(0.0, 1.0, (64, 3))
    Z = neutralise(rng.choice([-2, -1, 1, 2], 64), rng)
    quad = quad_spec("S", 59, n, L, True, b)
    dens = make_density(b, n, L, True, rng)
    boxes = np.array([[0, 0, 0, n, n, n]], np.int64)
    return System("cfg3", b, n, L, True, frac_to_pos(frac, b), Z, quad, dens, boxes, 140503)


def config4(count=512):
    rng = np.random.default_rng(140500 + 4)
    systems = []
    for i in range(count):
        b = 10.0
        Lv = int(rng.integers(4, 49))
        n = int(rng.choice([64, 96, 128, 192, 256]))
        M0 = int(rng.integers(1, 33))
        R = int(rng.choice([30, 36, 42, 48, 54, 60]))
        L = (Lv, Lv, Lv)
        frac = rng.uniform(0.0, 1.0, (M0, 3))
        Z = np.where(np.arange(M0) % 2 == 0, 1.0, -1.0)
        rng.shuffle(Z)
        quad = quad_spec("S", R - 1, n, L, False, b)
        dens = make_density(b, n, L, False, rng)
        o = (Lv // 2) * n
        boxes = np.array([[o, o, o, n, n, n]], np.int64)
        systems.append(System(f"cfg4[{i}]", b, n, L, False, frac_to_pos(frac, b), Z,
                              quad, dens, boxes, 140504))
    return systems


def config5():
    rng = np.random.default_rng(140500 + 5)
    b, n, L = 10.0, 128, (32, 32, 32)
    frac = rng.uniform(0.0, 1.0, (64, 3))
    Z = np.array([1.0] * 32 + [-1.0] * 32)
    rng.shuffle(Z)
    quad = quad_spec("S", 47, n, L, False, b)
    dens = make_density(b, n, L, False, rng)
    sysm = System("cfg5", b, n, L, False, frac_to_pos(frac, b), Z, quad, dens, None, 140505)
    sysm.extra["fd_step"] = 1e-4 * b
    return sysm


def small_box(seed, n=16, L=(3, 2, 3), M0=3, rule="S", M=29, neutral=True,
              on_grid=False, nbox=3, b=10.0, R_rho=8):
    """Oracle-sized box system of the same structure as the named workloads."""
    rng = np.random.default_rng(seed)
    if on_grid:
        frac = rng.integers(0, n, (M0, 3)) / n
    else:
        frac = rng.uniform(0.0, 1.0, (M0, 3))
    Z = rng.choice([-2.0, -1.0, 1.0, 2.0], M0)
    if neutral and M0 > 1:
        Z = neutralise(Z, rng)
    quad = quad_spec(rule, M, n, L, False, b)
    dens = make_density(b, n, L, False, rng, R_rho)
    N = [L[l] * n for l in range(3)]
    boxes = []
    for _ in range(nbox):
        e = [int(rng.integers(1, N[l] + 1)) for l in range(3)]
        o = [int(rng.integers(0, N[l] - e[l] + 1)) for l in range(3)]
        boxes.append(o + e)
    return System(f"small_box[{seed}]", b, n, tuple(L), False, frac_to_pos(frac, b), Z, quad,
                  dens, np.array(boxes, np.int64), seed)


def small_periodic(seed, n=16, L=(5, 5, 5), M0=4, rule="S", M=29, b=10.0, R_rho=8):
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0.0, 1.0, (M0, 3))
    Z = neutralise(rng.choice([-2.0, -1.0, 1.0, 2.0], M0), rng) if M0 > 1 else np.ones(1)
    quad = quad_spec(rule, M, n, L, True, b)
    dens = make_density(b, n, L, True, rng, R_rho)
    boxes = np.array([[0, 0, 0, n, n, n]], np.int64)
    return System(f"small_periodic[{seed}]", b, n, tuple(L), True, frac_to_pos(frac, b), Z, quad,
                  dens, boxes, seed)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make_basis(sysm, Nb, seed=7):
    """Nb separable Gaussian basis functions (rank one each) sampled at cell
    midpoints of the system's grid: centres at seeded atoms (with seeded
    offsets), exponents alpha ~ U[0.3, 3] / b^2 * n^0 (length^-2)."""
    rng = np.random.default_rng(seed)
    g = []
    atoms = rng.integers(0, sysm.M0, Nb)
    centres = sysm.pos[atoms] + rng.normal(0.0, 0.1 * sysm.b, (Nb, 3))
    alpha = rng.uniform(0.3, 3.0, Nb) / sysm.b ** 2 * 16.0
    for l in range(3):
        N = sysm.N(l)
        mid = -0.5 * sysm.b + (np.arange(N) + 0.5) * sysm.h
        g.append(np.exp(-alpha[:, None] * (mid[None, :] - centres[:, l, None]) ** 2))
    return g


def tensor_coords(rng, L, n, jitter, on_grid=False):
    """Lattice coordinates of one axis of a non-equidistant tensor lattice, in
    cells: k n plus a seeded displacement uniform in [-jitter, jitter] n per
    lattice plane (rounded to whole cells if ``on_grid``), sorted."""
    c = np.arange(L) * float(n) + rng.uniform(-jitter, jitter, L) * n
    c = np.sort(c - c.min())
    return np.rint(c) if on_grid else c


def _tensor_system(name, rng, b, n, L, frac, Z, M, jitter, on_grid, nbox, box_edge, seed):
    s = tuple(tensor_coords(rng, L[l], n, jitter, on_grid) for l in range(3))
    N = tuple(int(np.ceil(s[l][-1])) + n for l in range(3))
    C0, s_grid = rule_s_params(M, max(N))
    quad = {"rule": "S", "M": int(M), "C0": float(C0), "s": float(s_grid * n / b)}
    dens = make_density(b, n, L, False, rng, N=N)
    boxes = []
    for _ in range(nbox):
        e = [min(box_edge, N[l]) if box_edge else int(rng.integers(1, N[l] + 1)) for l in range(3)]
        o = [int(rng.integers(0, N[l] - e[l] + 1)) for l in range(3)]
        boxes.append(o + e)
    sysm = System(name, b, n, tuple(L), False, frac_to_pos(frac, b), Z, quad, dens,
                  np.array(boxes, np.int64), seed)
    sysm.extra["s"] = s
    sysm.extra["N"] = N
    return sysm


def small_tensor(seed, n=12, L=(3, 2, 4), M0=3, jitter=0.3, on_grid=False, nbox=3, b=10.0):
    """Oracle-sized non-equidistant tensor lattice (lattice coordinates in
    extra["s"], grid cells per axis in extra["N"])."""
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0.0, 1.0, (M0, 3))
    Z = neutralise(rng.choice([-2.0, -1.0, 1.0, 2.0], M0), rng) if M0 > 1 else np.ones(1)
    return _tensor_system(f"small_tensor[{seed}]", rng, b, n, L, frac, Z, 29, jitter, on_grid,
                          nbox, 0, seed)


def config_tensor():
    """The headline structure on a non-equidistant tensor lattice: 32 lattice
    planes per axis at k n + U[-0.25, 0.25] n cells (n = 128, b = 10), the
    8-site rock-salt cell of the box workload, rule S R=48, 16 sub-boxes of
    256^3 cells, rank-8 density."""
    rng = np.random.default_rng(140500 + 6)
    b, n, L = 10.0, 128, (32, 32, 32)
    A = [(.25, .25, .25), (.25, .75, .75), (.75, .25, .75), (.75, .75, .25)]
    B = [(.75, .75, .75), (.75, .25, .25), (.25, .75, .25), (.25, .25, .75)]
    frac = np.array(A + B) + rng.uniform(-0.05, 0.05, (8, 3))
    Z = np.array([1.0] * 4 + [-1.0] * 4)
    return _tensor_system("cfg_tensor", rng, b, n, L, frac, Z, 47, 0.25, False, 16, 256, 140506)


def config_slab(L, n=128, slab=True):
    """Table 3.1's lattices of unit charges: L x L x 1 (slab) or L x L x L, one
    charge at the centre of each cell (b = 10, n cells per edge), rule S R=48."""
    b = 10.0
    Ls = (L, L, 1) if slab else (L, L, L)
    pos = frac_to_pos([[0.5, 0.5, 0.5]], b)
    quad = quad_spec("S", 47, n, Ls, False, b)
    return System(f"slab[{L}]" if slab else f"cube[{L}]", b, n, Ls, False, pos, np.array([1.0]),
                  quad, None, None, 140507)
