"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the method: it only writes down lattices
(site numbering, periodic nearest-neighbour bond lists, couplings) and seeded
random draws.  Both the HIP library and the CPU oracle receive what it returns
as plain arrays.

Site numbering: site i <-> (x, y, z) with i = x + Lx*(y + Ly*z), all 0-based;
with S sites per unit cell (kagome, honeycomb), i = s + S*(x + Lx*(y + Ly*z))
for sublattice s of cell (x, y, z).
A bond is (i, j, Jxy, Jz) with the XXZ convention of the paper's model
(Sec. 2.2): J > 0 is antiferromagnetic.
"""
from __future__ import annotations

import dataclasses
import itertools
import numpy as np


@dataclasses.dataclass(frozen=True)
class Lattice:
    name: str
    lx: int
    ly: int
    lz: int
    bi: np.ndarray      # int32 [n_bonds]
    bj: np.ndarray      # int32 [n_bonds]
    jxy: np.ndarray     # float64 [n_bonds]
    jz: np.ndarray      # float64 [n_bonds]
    translation_invariant: bool = True
    ns: int = 1         # sites per unit cell
    basis: tuple = ()   # positions of the places in a cell (cell-vector units), () = all at 0

    @property
    def n_sites(self) -> int:
        return self.ns * self.lx * self.ly * self.lz

    @property
    def n_bonds(self) -> int:
        return int(self.bi.shape[0])

    @property
    def dims(self) -> tuple:
        return (self.lx, self.ly, self.lz)


def site_index(x: int, y: int, z: int, lx: int, ly: int) -> int:
    return x + lx * (y + ly * z)


def hypercubic(lx: int, ly: int = 1, lz: int = 1, J: float = 1.0, Delta: float = 1.0,
               name: str | None = None) -> Lattice:
    """Periodic nearest-neighbour bonds on an lx x ly x lz lattice.

    Each site gets one bond in each direction whose length is > 1 (a length-2
    direction would otherwise give the same bond twice; length 2 keeps one).
    """
    bonds = []
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                i = site_index(x, y, z, lx, ly)
                for (L, nb) in ((lx, ((x + 1) % lx, y, z)), (ly, (x, (y + 1) % ly, z)),
                                (lz, (x, y, (z + 1) % lz))):
                    if L == 1:
                        continue
                    bonds.append((i, site_index(nb[0], nb[1], nb[2], lx, ly)))
    # drop duplicate undirected bonds (length-2 directions)
    seen = set()
    uniq = []
    for (i, j) in bonds:
        key = (min(i, j), max(i, j))
        if key in seen:
            continue
        seen.add(key)
        uniq.append(key)
    bi = np.array([b[0] for b in uniq], dtype=np.int32)
    bj = np.array([b[1] for b in uniq], dtype=np.int32)
    nb = len(uniq)
    if name is None:
        name = f"hypercubic{lx}x{ly}x{lz}"
    return Lattice(name, lx, ly, lz, bi, bj,
                   np.full(nb, float(J)), np.full(nb, float(J) * float(Delta)), True)


def chain(L: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    return hypercubic(L, 1, 1, J, Delta, name=f"chain{L}")


def square(L: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    return hypercubic(L, L, 1, J, Delta, name=f"square{L}x{L}")


def square_j1j2(L: int, J2: float, Delta: float = 1.0) -> Lattice:
    """Periodic L x L square (L >= 3) with J1 = 1 on the edges and J2 on both
    diagonals of every plaquette: two exchange constants, the C4v symmetry
    of the square kept."""
    base = square(L, 1.0, Delta)
    di, dj = [], []
    for y in range(L):
        for x in range(L):
            for dy in (1, -1):
                di.append(x + L * y)
                dj.append((x + 1) % L + L * ((y + dy) % L))
    n = len(di)
    return dataclasses.replace(base, name=f"square{L}x{L}+j2", bi=np.concatenate([base.bi, np.array(di, np.int32)]),
                               bj=np.concatenate([base.bj, np.array(dj, np.int32)]),
                               jxy=np.concatenate([base.jxy, np.full(n, J2)]),
                               jz=np.concatenate([base.jz, np.full(n, J2 * Delta)]))


def cube(L: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    return hypercubic(L, L, L, J, Delta, name=f"cube{L}^3")


def _cell_lattice(name: str, ns: int, lx: int, ly: int, links, J: float, Delta: float,
                  basis: tuple = (), lz: int = 1) -> Lattice:
    """Periodic lx x ly x lz cells of ns sites; links: (s, t, dx, dy) or
    (s, t, dx, dy, dz) couples sublattice s of cell (x, y, z) with sublattice
    t of cell (x + dx, y + dy, z + dz)."""
    seen = set()
    uniq = []
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                for link in links:
                    s, t, dx, dy = link[:4]
                    dz = link[4] if len(link) > 4 else 0
                    i = s + ns * site_index(x, y, z, lx, ly)
                    j = t + ns * site_index((x + dx) % lx, (y + dy) % ly, (z + dz) % lz, lx, ly)
                    key = (min(i, j), max(i, j))
                    if i == j or key in seen:
                        continue
                    seen.add(key)
                    uniq.append(key)
    bi = np.array([b[0] for b in uniq], dtype=np.int32)
    bj = np.array([b[1] for b in uniq], dtype=np.int32)
    nb = len(uniq)
    return Lattice(name, lx, ly, lz, bi, bj, np.full(nb, float(J)), np.full(nb, float(J) * float(Delta)),
                   True, ns, basis)


def kagome(lx: int, ly: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    """Kagome lattice: triangular Bravais lattice (a1, a2) with sublattices
    0 at 0, 1 at a1/2, 2 at a2/2; each site has 4 neighbours (two up and two
    down triangles).  Needs lx, ly >= 2."""
    links = [(0, 1, 0, 0), (0, 2, 0, 0), (1, 2, 0, 0),      # up triangle of the cell
             (1, 0, 1, 0), (2, 0, 0, 1), (1, 2, 1, -1)]     # down triangles
    return _cell_lattice(f"kagome{lx}x{ly}", 3, lx, ly, links, J, Delta,
                         ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0)))


def honeycomb(lx: int, ly: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    """Honeycomb lattice: two sublattices, each site with 3 neighbours."""
    links = [(0, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1)]
    return _cell_lattice(f"honeycomb{lx}x{ly}", 2, lx, ly, links, J, Delta,
                         ((0.0, 0.0, 0.0), (1.0 / 3.0, 1.0 / 3.0, 0.0)))


def pyrochlore(L: int, J: float = 1.0, Delta: float = 1.0) -> Lattice:
    """Pyrochlore lattice: fcc Bravais lattice (a1, a2, a3) with a tetrahedron
    of four sublattices, 0 at the cell's origin and s = 1..3 at a_s / 2; every
    site has 6 neighbours (three in the cell's up tetrahedron, three in a down
    tetrahedron: sublattice s of cell R with 0 of R + a_s and with t of
    R + a_s - a_t).  L x L x L cells, L >= 2."""
    up = [(s, t, 0, 0, 0) for s in range(4) for t in range(s + 1, 4)]
    e = {1: (1, 0, 0), 2: (0, 1, 0), 3: (0, 0, 1)}
    down = [(s, 0) + e[s] for s in (1, 2, 3)]
    down += [(s, t) + tuple(a - b for a, b in zip(e[s], e[t])) for s in (1, 2, 3) for t in (1, 2, 3) if s < t]
    return _cell_lattice(f"pyrochlore{L}^3", 4, L, L, up + down, J, Delta,
                         ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5)), lz=L)


def with_disorder(lat: Lattice, seed: int, jlo: float = 0.5, jhi: float = 1.5,
                  dlo: float = 0.0, dhi: float = 2.0, per_bond: bool = True) -> Lattice:
    """Bond disorder of the serving stream: J_ij ~ U[jlo, jhi] per bond (or one J
    for all bonds when per_bond is False), Delta ~ U[dlo, dhi] once per request."""
    rng = np.random.default_rng(seed)
    if per_bond:
        J = rng.uniform(jlo, jhi, size=lat.n_bonds)
    else:
        J = np.full(lat.n_bonds, rng.uniform(jlo, jhi))
    Delta = rng.uniform(dlo, dhi)
    return dataclasses.replace(lat, name=lat.name + f"+dis{seed}", jxy=J.astype(np.float64),
                               jz=(J * Delta).astype(np.float64),
                               translation_invariant=(not per_bond))


def random_bonds(n_sites: int, n_bonds: int, seed: int) -> Lattice:
    """A random bond graph (no translation symmetry) with random couplings."""
    rng = np.random.default_rng(seed)
    seen = set()
    out = []
    while len(out) < n_bonds:
        i, j = rng.integers(0, n_sites, size=2)
        if i == j:
            continue
        key = (int(min(i, j)), int(max(i, j)))
        if key in seen:
            continue
        seen.add(key)
        out.append(key)
    bi = np.array([b[0] for b in out], dtype=np.int32)
    bj = np.array([b[1] for b in out], dtype=np.int32)
    return Lattice(f"random{n_sites}_{n_bonds}_{seed}", n_sites, 1, 1, bi, bj,
                   rng.uniform(-1.0, 1.5, size=n_bonds), rng.uniform(-1.0, 2.0, size=n_bonds),
                   False)


# one-dimensional representations of C4v on the operations of c4v_ops, in its
# order (identity, rotations by 90, 180, 270 degrees, mirrors x -> -x and
# y -> -y, diagonal mirrors (x, y) -> (y, x) and (-y, -x))
C4V_CHARS = {"A1": (1, 1, 1, 1, 1, 1, 1, 1), "A2": (1, 1, 1, 1, -1, -1, -1, -1),
             "B1": (1, -1, 1, -1, 1, 1, -1, -1), "B2": (1, -1, 1, -1, -1, -1, 1, 1)}
# the two-dimensional one (characters only; no basis is built for it)
C4V_E = (2, 0, -2, 0, 0, 0, 0, 0)


def c4v_ops(L: int) -> np.ndarray:
    """The point group C4v of the periodic L x L square about site 0, as site
    permutations perm[p][i] (int32, 8 x L^2)."""
    maps = [lambda x, y: (x, y), lambda x, y: (-y, x), lambda x, y: (-x, -y), lambda x, y: (y, -x),
            lambda x, y: (-x, y), lambda x, y: (x, -y), lambda x, y: (y, x), lambda x, y: (-y, -x)]
    out = np.zeros((8, L * L), dtype=np.int32)
    for p, f in enumerate(maps):
        for y in range(L):
            for x in range(L):
                u, v = f(x, y)
                out[p, x + L * y] = (u % L) + L * (v % L)
    return out


def inversion_ops(L: int) -> np.ndarray:
    """Identity and the inversion x -> -x of the periodic chain (2 x L)."""
    return np.array([[i for i in range(L)], [(-i) % L for i in range(L)]], dtype=np.int32)


def honeycomb_inversion_ops(lx: int, ly: int) -> np.ndarray:
    """Identity and the inversion through the centre of the bond A(0)-B(0) of
    the honeycomb lattice (workloads.honeycomb): A at R <-> B at -R, which
    exchanges the two places of a cell (2 x 2 lx ly)."""
    N = 2 * lx * ly
    out = np.zeros((2, N), dtype=np.int32)
    out[0] = np.arange(N)
    for y in range(ly):
        for x in range(lx):
            c, cm = x + lx * y, ((-x) % lx) + lx * ((-y) % ly)
            out[1, 2 * c] = 1 + 2 * cm
            out[1, 2 * c + 1] = 2 * cm
    return out


def kagome_c6v_ops(L: int) -> np.ndarray:
    """C6v of the periodic L x L kagome lattice (workloads.kagome) about a
    hexagon centre, as site permutations (12 x 3 L^2): R^k then R^k M for
    k = 0..5, R the 60-degree rotation and M the mirror exchanging a1 and a2.
    In doubled coordinates on (a1, a2) the places sit at 2(x, y) + (0, 0),
    (1, 0), (0, 1), the centre at (1, 1); R: (u, v) -> (-v, u + v)."""
    d = ((0, 0), (1, 0), (0, 1))

    def site_of(u, v):
        u %= 2 * L
        v %= 2 * L
        for s, (dx, dy) in enumerate(d):
            if (u - dx) % 2 == 0 and (v - dy) % 2 == 0:
                return s + 3 * ((u - dx) // 2 + L * ((v - dy) // 2))
        raise ValueError("not a kagome site")

    out = np.zeros((12, 3 * L * L), dtype=np.int32)
    for m in (0, 1):
        for k in range(6):
            for i in range(3 * L * L):
                s, c = i % 3, i // 3
                u, v = 2 * (c % L) + d[s][0] - 1, 2 * (c // L) + d[s][1] - 1
                if m:
                    u, v = v, u
                for _ in range(k):
                    u, v = -v, u + v
                out[6 * m + k, i] = site_of(u + 1, v + 1)
    return out


def honeycomb_c6v_ops(L: int) -> np.ndarray:
    """C6v of the periodic L x L honeycomb lattice (workloads.honeycomb) about
    a hexagon centre, in the order of kagome_c6v_ops.  In tripled coordinates
    on (a1, a2) the places sit at 3(x, y) and 3(x, y) + (1, 1), the centre at
    (2, 2); R: (u, v) -> (-v, u + v), M: (u, v) -> (v, u)."""
    d = ((0, 0), (1, 1))

    def site_of(u, v):
        u %= 3 * L
        v %= 3 * L
        for s, (dx, dy) in enumerate(d):
            if (u - dx) % 3 == 0 and (v - dy) % 3 == 0:
                return s + 2 * ((u - dx) // 3 + L * ((v - dy) // 3))
        raise ValueError("not a honeycomb site")

    out = np.zeros((12, 2 * L * L), dtype=np.int32)
    for m in (0, 1):
        for k in range(6):
            for i in range(2 * L * L):
                s, c = i % 2, i // 2
                u, v = 3 * (c % L) + d[s][0] - 2, 3 * (c // L) + d[s][1] - 2
                if m:
                    u, v = v, u
                for _ in range(k):
                    u, v = -v, u + v
                out[6 * m + k, i] = site_of(u + 2, v + 2)
    return out


# one-dimensional characters of C6v in the order of kagome_c6v_ops and
# honeycomb_c6v_ops
C6V_CHARS = {"A1": (1,) * 12, "A2": (1,) * 6 + (-1,) * 6,
             "B1": tuple((-1) ** k for k in range(6)) * 2,
             "B2": tuple((-1) ** k for k in range(6)) + tuple(-((-1) ** k) for k in range(6))}


def _oh_elements():
    """The 48 signed axis permutations (sigma, signs) of O_h, identity first."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            out.append((perm, signs))
    out.sort(key=lambda e: (e[0] != (0, 1, 2) or e[1] != (1, 1, 1)))
    return out


def _perm_sign(perm) -> int:
    inv = sum(1 for i in range(3) for j in range(i + 1, 3) if perm[i] > perm[j])
    return -1 if inv % 2 else 1


def oh_ops(L: int) -> np.ndarray:
    """The point group O_h of the periodic L x L x L cube about site 0 as site
    permutations (48 x L^3): (x_0, x_1, x_2) -> (s_a x_{sigma(a)})_a mod L."""
    els = _oh_elements()
    out = np.zeros((len(els), L ** 3), dtype=np.int32)
    for p, (perm, signs) in enumerate(els):
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    r = (x, y, z)
                    img = [(signs[a] * r[perm[a]]) % L for a in range(3)]
                    out[p, x + L * (y + L * z)] = img[0] + L * (img[1] + L * img[2])
    return out


def oh_chars() -> dict:
    """Characters of the four one-dimensional representations of O_h in the
    order of oh_ops: A1g 1, A2g sign(sigma), A1u det, A2u sign(sigma) det
    (det = sign(sigma) times the product of the signs)."""
    out = {"A1g": [], "A2g": [], "A1u": [], "A2u": []}
    for perm, signs in _oh_elements():
        ps = _perm_sign(perm)
        det = ps * signs[0] * signs[1] * signs[2]
        out["A1g"].append(1)
        out["A2g"].append(ps)
        out["A1u"].append(det)
        out["A2u"].append(ps * det)
    return {k: tuple(v) for k, v in out.items()}


def all_momenta(lat: Lattice) -> list:
    """Every momentum index triple (Kx, Ky, Kz), Kx fastest."""
    out = []
    for kz in range(lat.lz):
        for ky in range(lat.ly):
            for kx in range(lat.lx):
                out.append((kx, ky, kz))
    return out


def serving_stream(n_requests: int, seed: int, rate: float):
    """Poisson arrivals of solve requests for the serving workload.

    Lattice family uniform over {chain L in [16,64], square L in [6,12],
    cube L in [6,10]}, all periodic; N_down uniform in {1..4}; with a momentum
    sector with probability 1/2.  With a momentum sector the couplings are one
    J ~ U[0.5,1.5] for all bonds (disorder would break translation symmetry);
    without, J_ij ~ U[0.5,1.5] per bond; Delta ~ U[0,2] once per request.
    Returns a list of dicts with arrival times in seconds.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        fam = int(rng.integers(0, 3))
        if fam == 0:
            L = int(rng.integers(16, 65)); lat = chain(L)
        elif fam == 1:
            L = int(rng.integers(6, 13)); lat = square(L)
        else:
            L = int(rng.integers(6, 11)); lat = cube(L)
        n_down = int(rng.integers(1, 5))
        use_k = bool(rng.integers(0, 2))
        lat = with_disorder(lat, seed=int(rng.integers(0, 2**31)), per_bond=not use_k)
        K = None
        if use_k:
            K = (int(rng.integers(0, lat.lx)), int(rng.integers(0, lat.ly)), int(rng.integers(0, lat.lz)))
        reqs.append(dict(id=r, t_arrive=t, lattice=lat, n_down=n_down, K=K))
    return reqs
