"""Synthetic system definitions, plane-wave spheres and seeded random inputs.

Units are Hartree atomic units (bohr, Ha).  The paper works in Hartree units
(Sec. 2.1) and runs on a CrI3 monolayer with norm-conserving pseudopotentials
(Sec. 5.1); those pseudopotentials are not available, so the systems below
are synthetic stand-ins with the same ingredients: a local potential per
atom, Kleinman-Bylander projectors and a spin-orbit D matrix that commutes
with time reversal (Sec. 2.2, the statement that the nonlocal SOC term is
time-reversal invariant).

Conventions fixed here (they define the inputs, not the method):

* ``cell`` rows are the lattice vectors a1, a2, a3; ``recip`` rows are b_i
  with a_i . b_j = 2 pi delta_ij; G = m1 b1 + m2 b2 + m3 b3 for integer
  Miller indices m.
* Real-space grid point (i1, i2, i3) sits at r = (i1/n1) a1 + (i2/n2) a2 +
  (i3/n3) a3; grid arrays are numpy C-order with shape (n1, n2, n3).
* A plane-wave sphere at k is {G : |k+G|^2 / 2 < ecut}, sorted by (m1, m2, m3)
  so that each (m1, m2) column is contiguous.
* Spinor coefficient arrays are laid out [band][spin][G] (spin 0 = up).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Atom", "SystemDef", "recip", "volume", "sphere", "grid_points",
    "vloc_grid", "projector_table", "dmatrix", "make_cubic20", "make_tiny",
    "make_hexslab", "kmesh_cart", "QSetDef", "qset_exact", "qset_folded",
    "random_br", "synthetic_ground_state", "synthetic_fields", "synthetic_inputs",
    "cart_from_frac", "q_path", "synthetic_inputs_multi", "make_cubic",
]


@dataclass
class Atom:
    pos: np.ndarray            # Cartesian position (bohr)
    depth: float               # depth A of the Gaussian well -A exp(-r^2/2w^2) (Ha)
    width: float               # Gaussian width w (bohr)
    kinds: Tuple[str, ...]     # projector kinds: 's', 'px', 'py'
    dscal: Tuple[float, ...]   # scalar (spin-diagonal) D entry per projector (Ha)
    soc: float = 0.0           # coupling i*soc*sigma_z between the px and py projectors


@dataclass
class SystemDef:
    name: str
    cell: np.ndarray
    atoms: List[Atom]
    ecut: float                # wavefunction cutoff, |k+G|^2/2 < ecut (Ha)
    fft: Tuple[int, int, int]
    nbnd: int                  # occupied spinor bands (fixed integer occupation)
    kmesh: np.ndarray          # SCF k-mesh in crystal coordinates, shape [nk][3]
    seed: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def recip(self) -> np.ndarray:
        return recip(self.cell)

    @property
    def omega(self) -> float:
        return volume(self.cell)

    @property
    def nproj(self) -> int:
        return sum(len(a.kinds) for a in self.atoms)

    @property
    def ngrid(self) -> int:
        return int(np.prod(self.fft))


def recip(cell: np.ndarray) -> np.ndarray:
    return 2.0 * np.pi * np.linalg.inv(np.asarray(cell, dtype=float)).T


def volume(cell: np.ndarray) -> float:
    return float(abs(np.linalg.det(np.asarray(cell, dtype=float))))


def cart_from_frac(sysd: SystemDef, frac) -> np.ndarray:
    """Crystal (fractional reciprocal) coordinates -> Cartesian k (bohr^-1)."""
    return np.asarray(frac, dtype=float) @ sysd.recip


def kmesh_cart(sysd: SystemDef) -> np.ndarray:
    return cart_from_frac(sysd, sysd.kmesh)


def sphere(sysd: SystemDef, kcart, ecut: float | None = None) -> np.ndarray:
    """Miller indices [npw][3] (int32) of the sphere |k+G|^2/2 < ecut, column-sorted."""
    ecut = sysd.ecut if ecut is None else ecut
    b = sysd.recip
    k = np.asarray(kcart, dtype=float)
    gmax = np.sqrt(2.0 * ecut) + np.linalg.norm(k)
    # |m_i| <= gmax * |a_i| / (2 pi) bounds every component of the sphere
    lim = [int(np.ceil(gmax * np.linalg.norm(sysd.cell[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-l, l + 1) for l in lim]
    m = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    kg = k + m @ b
    keep = 0.5 * np.einsum("ij,ij->i", kg, kg) < ecut
    m = m[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0]))
    m = m[order].astype(np.int32)
    n = np.asarray(sysd.fft)
    if np.any(2 * np.abs(m) >= n):
        raise ValueError("sphere does not fit in the FFT grid")
    return m


def grid_points(sysd: SystemDef) -> np.ndarray:
    """Cartesian coordinates of the grid points, shape (n1, n2, n3, 3)."""
    n1, n2, n3 = sysd.fft
    f = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2,
                             np.arange(n3) / n3, indexing="ij"), axis=-1)
    return f @ sysd.cell


def _image_sum(sysd: SystemDef, func, images=(2, 2, 2)) -> np.ndarray:
    """Sum of func(|r - R - L|^2, atom) over atoms and periodic images L."""
    n1, n2, n3 = sysd.fft
    frac = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2,
                                np.arange(n3) / n3, indexing="ij"), axis=-1).reshape(-1, 3)
    inv = np.linalg.inv(sysd.cell)
    out = np.zeros(frac.shape[0])
    for at in sysd.atoms:
        fa = at.pos @ inv
        d0 = frac - fa
        d0 -= np.round(d0)  # minimum image in crystal coordinates
        for i in range(-images[0], images[0] + 1):
            for j in range(-images[1], images[1] + 1):
                for l in range(-images[2], images[2] + 1):
                    d = (d0 + np.array([i, j, l])) @ sysd.cell
                    out += func(np.einsum("ij,ij->i", d, d), at)
    return out.reshape(n1, n2, n3)


def vloc_grid(sysd: SystemDef) -> np.ndarray:
    """Local potential sum_R -A exp(-|r-R|^2 / 2w^2), sampled on the grid (Ha)."""
    return _image_sum(sysd, lambda r2, at: -at.depth * np.exp(-r2 / (2 * at.width ** 2)))


def projector_table(sysd: SystemDef, kcart, mill: np.ndarray) -> np.ndarray:
    """beta_i(k+G) = Omega^{-1/2} int exp(-i(k+G).r) beta_i(r) dr, shape [nproj][npw].

    The real-space projectors are real: s = N_s g(r), px = N_p x g(r),
    py = N_p y g(r), g = exp(-r^2/2w^2) centred on the atom, each normalised
    to int |beta|^2 = 1.
    """
    K = np.asarray(kcart, dtype=float) + mill @ sysd.recip
    k2 = np.einsum("ij,ij->i", K, K)
    rows = []
    pref = 1.0 / np.sqrt(sysd.omega)
    for at in sysd.atoms:
        w = at.width
        gauss = (2 * np.pi * w * w) ** 1.5 * np.exp(-0.5 * k2 * w * w)
        phase = np.exp(-1j * (K @ at.pos))
        for kind in at.kinds:
            if kind == "s":
                ns = (np.pi ** 1.5 * w ** 3) ** -0.5
                rows.append(pref * ns * gauss * phase)
            elif kind in ("px", "py"):
                npn = (np.pi ** 1.5 * w ** 5 / 2.0) ** -0.5
                comp = K[:, 0] if kind == "px" else K[:, 1]
                rows.append(pref * npn * (-1j) * comp * w * w * gauss * phase)
            else:
                raise ValueError(kind)
    return np.array(rows, dtype=np.complex128).reshape(len(rows), K.shape[0])


def dmatrix(sysd: SystemDef) -> np.ndarray:
    """Spinor D matrix [nproj][nproj][2][2] (Ha), block diagonal in atoms.

    D_ij = a_ij sigma_0 + i c_ij . sigma with a real symmetric and c real
    antisymmetric, which is the form that commutes with time reversal for
    real projectors.  Here a is diagonal (dscal) and c couples px and py of
    the same atom along z with strength ``soc``.
    """
    n = sysd.nproj
    d = np.zeros((n, n, 2, 2), dtype=np.complex128)
    s0 = np.eye(2)
    sz = np.diag([1.0, -1.0])
    off = 0
    for at in sysd.atoms:
        for i, val in enumerate(at.dscal):
            d[off + i, off + i] = val * s0
        if at.soc != 0.0 and "px" in at.kinds and "py" in at.kinds:
            ix = off + at.kinds.index("px")
            iy = off + at.kinds.index("py")
            d[ix, iy] = 1j * at.soc * sz
            d[iy, ix] = -1j * at.soc * sz
        off += len(at.kinds)
    return d


def _random_positions(rng, cell, nat, min_sep):
    while True:
        frac = rng.random((nat, 3))
        ok = True
        for i in range(nat):
            for j in range(i):
                d = frac[i] - frac[j]
                d -= np.round(d)
                if np.linalg.norm(d @ cell) < min_sep:
                    ok = False
        if ok:
            return frac @ cell


def make_cubic20(seed: int = 2205, soc: float = 0.01, nbnd: int = 8) -> SystemDef:
    """Oracle-sized cubic system: a = 10 bohr, 2 atoms, ~500 PW, 20^3 grid, Gamma.

    Seed 2205 is the first seed from 2203 upward whose SCF ground state has a
    HOMO-LUMO gap >= 0.02 Ha (2203 gives 0.019 Ha, 2204 0.010 Ha).
    """
    rng = np.random.default_rng(seed)
    a = 10.0
    cell = a * np.eye(3)
    pos = _random_positions(rng, cell, 2, 3.0)
    atoms = []
    for p in pos:
        depth = rng.uniform(2.0, 4.0)
        width = rng.uniform(0.8, 1.2)
        d = rng.uniform(0.2, 0.5)
        atoms.append(Atom(pos=p, depth=depth, width=width, kinds=("px", "py"),
                          dscal=(d, d), soc=soc))
    ecut = 4.79
    return SystemDef(name="cubic20", cell=cell, atoms=atoms, ecut=ecut, fft=(20, 20, 20),
                     nbnd=nbnd, kmesh=np.zeros((1, 3)), seed=seed)


def make_cubic(n: int, nbnd: int, mesh: int, seed: int = 2205, soc: float = 0.01) -> SystemDef:
    """cubic20's cell and atoms on an n^3 grid: E_cut scaled with n^2 (so the
    sphere fills the grid as at 20^3), nbnd bands, Gamma-centred mesh x mesh x 1."""
    base = make_cubic20(seed=seed, soc=soc, nbnd=nbnd)
    f = np.arange(mesh) / mesh
    kmesh = np.array([[a, b, 0.0] for a in f for b in f])
    return SystemDef(name=f"cubic{n}", cell=base.cell, atoms=base.atoms, ecut=base.ecut * (n / 20.0) ** 2,
                     fft=(n, n, n), nbnd=nbnd, kmesh=kmesh, seed=seed)


def make_tiny(seed: int = 7, nat: int = 2, a: float = 6.0, ecut: float = 2.0,
              fft=(8, 8, 8), nbnd: int = 3, soc: float = 0.01,
              kmesh=((0.0, 0.0, 0.0),), kinds=("px", "py"),
              depth=(2.0, 4.0), width=(0.8, 1.2)) -> SystemDef:
    """Tiny cubic system for dense-matrix checks (a few dozen plane waves)."""
    rng = np.random.default_rng(seed)
    cell = a * np.eye(3)
    pos = _random_positions(rng, cell, nat, min(2.5, a / 3))
    atoms = []
    for p in pos:
        dep = rng.uniform(*depth)
        wid = rng.uniform(*width)
        d = rng.uniform(0.2, 0.5)
        atoms.append(Atom(pos=p, depth=dep, width=wid, kinds=tuple(kinds),
                          dscal=tuple(d for _ in kinds), soc=soc))
    return SystemDef(name="tiny", cell=cell, atoms=atoms, ecut=ecut, fft=tuple(fft),
                     nbnd=nbnd, kmesh=np.asarray(kmesh, dtype=float), seed=seed)


# In-plane crystal coordinates of a honeycomb MX3 layer (2 metal + 6 halogen
# sites) and the heights of the three atomic planes relative to the metal
# plane, in bohr.  This is the structural pattern of a CrI3 monolayer.
_CRI3_SITES = [
    ("Cr", 0.6666667, 0.3333333, 0.0),
    ("Cr", 0.0000000, 0.0000000, 0.0),
    ("I", 0.9788986, 0.6665119, +2.98),
    ("I", 0.6876134, 0.0211013, +2.98),
    ("I", 0.3334880, 0.3123867, +2.98),
    ("I", 0.6877680, 0.6668213, -2.98),
    ("I", 0.9790533, 0.3122319, -2.98),
    ("I", 0.3331787, 0.0209467, -2.98),
]


def make_hexslab(seed: int = 2022, a: float = 13.0, c: float = 31.0, ecut: float = 11.09,
              fft=(48, 48, 180), nbnd: int = 104, nk: int = 6, soc: float = 0.02) -> SystemDef:
    """CrI3-monolayer-shaped hexagonal slab: 2 'Cr' + 6 'I', 6x6x1 Gamma-centred mesh."""
    rng = np.random.default_rng(seed)
    cell = np.array([[a, 0, 0], [-0.5 * a, 0.5 * np.sqrt(3) * a, 0], [0, 0, c]])
    atoms = []
    for name, f1, f2, dz in _CRI3_SITES:
        p = np.array([f1, f2, 0.5]) @ cell + np.array([0, 0, dz])
        if name == "Cr":
            depth = rng.uniform(3.0, 4.0)
            lam = 0.0
        else:
            depth = rng.uniform(2.0, 3.0)
            lam = soc
        width = rng.uniform(0.8, 1.2)
        d = rng.uniform(0.2, 0.5, size=3)
        atoms.append(Atom(pos=p, depth=depth, width=width, kinds=("s", "px", "py"),
                          dscal=tuple(d), soc=lam))
    km = np.array([[i / nk, j / nk, 0.0] for i in range(nk) for j in range(nk)])
    return SystemDef(name="hexslab", cell=cell, atoms=atoms, ecut=ecut, fft=tuple(fft),
                     nbnd=nbnd, kmesh=km, seed=seed, notes={"c": c, "vacuum": c - 6.0})


@dataclass
class QSetDef:
    """The k-related points of one q: for every mesh k the points k, -k, k+q, -k-q.

    ``points`` holds the distinct Cartesian vectors that carry ground-state
    data; ``roles[ik] = (ik_k, ik_mk, ik_kq, ik_mkq)`` index into it and
    ``shifts[ik][role]`` is the integer Miller vector g with
    (role vector) = points[index] + g . recip.
    """
    q: np.ndarray
    kmesh: np.ndarray
    points: np.ndarray
    roles: np.ndarray
    shifts: np.ndarray


def qset_exact(sysd: SystemDef, qcart, bitwise: bool = False) -> QSetDef:
    """Every role vector kept as its own point (no folding).

    With bitwise=True two role vectors share a point only if they are equal
    bit for bit, so -k-q is always the exact negation of k+q and the two
    spheres are exact negatives of each other.
    """
    q = np.asarray(qcart, dtype=float)
    km = kmesh_cart(sysd)
    pts: list = []

    def idx(v):
        for i, p in enumerate(pts):
            if (np.array_equal(p, v) if bitwise else np.allclose(p, v, atol=1e-12)):
                return i
        pts.append(np.array(v, dtype=float))
        return len(pts) - 1

    roles = []
    for k in km:
        roles.append([idx(k), idx(-k), idx(k + q), idx(-k - q)])
    nk = len(km)
    return QSetDef(q=q, kmesh=km, points=np.array(pts), roles=np.array(roles, dtype=np.int32),
                   shifts=np.zeros((nk, 4, 3), dtype=np.int32))


def qset_folded(sysd: SystemDef, qfrac) -> QSetDef:
    """Role vectors folded onto the mesh itself (q must be a mesh vector)."""
    qf = np.asarray(qfrac, dtype=float)
    mesh = np.asarray(sysd.kmesh, dtype=float)

    def find(vf):
        for i, m in enumerate(mesh):
            d = vf - m
            if np.allclose(d, np.round(d), atol=1e-9):
                return i, np.round(d).astype(np.int32)
        raise ValueError("point not on the mesh")

    roles, shifts = [], []
    for kf in mesh:
        r, s = zip(*[find(v) for v in (kf, -kf, kf + qf, -kf - qf)])
        roles.append(r)
        shifts.append(s)
    return QSetDef(q=qf @ sysd.recip, kmesh=mesh @ sysd.recip, points=mesh @ sysd.recip,
                   roles=np.array(roles, dtype=np.int32), shifts=np.array(shifts, dtype=np.int32))


def random_br(nk: int, nb: int, npw: Sequence[int], npw_pad: int, seed: int) -> np.ndarray:
    """Seeded random BR vector [2][nk][nb][2][npw_pad] with zero padding."""
    rng = np.random.default_rng(seed)
    v = np.zeros((2, nk, nb, 2, npw_pad), dtype=np.complex128)
    for s in range(2):
        for ik in range(nk):
            n = npw[ik]
            v[s, ik, :, :, :n] = rng.standard_normal((nb, 2, n)) + 1j * rng.standard_normal((nb, 2, n))
    return v


def synthetic_ground_state(sysd: SystemDef, kcart, mill, seed: int, sigma2: float = 4.0):
    """Smooth random orthonormal occupied spinors [nb][2][npw] and eigenvalues.

    Used only for benchmark shapes where a self-consistent ground state is too
    expensive to produce: coefficients are complex Gaussians damped by
    exp(-|k+G|^2 / (2 sigma2)) and orthonormalised.  Eigenvalues are placed
    well below the bottom of the local potential so that the diagonal part of
    the Liouvillian stays positive.
    """
    rng = np.random.default_rng(seed)
    nb = sysd.nbnd
    K = np.asarray(kcart, dtype=float) + mill @ sysd.recip
    damp = np.exp(-0.5 * np.einsum("ij,ij->i", K, K) / sigma2)
    npw = mill.shape[0]
    a = (rng.standard_normal((2 * npw, nb)) + 1j * rng.standard_normal((2 * npw, nb)))
    a *= np.concatenate([damp, damp])[:, None]
    qm, _ = np.linalg.qr(a)
    evc = np.ascontiguousarray(qm.T.reshape(nb, 2, npw))
    vmin = -max(at.depth for at in sysd.atoms)
    et = np.sort(vmin - 1.5 + 0.5 * rng.random(nb))
    return evc, et


def synthetic_inputs(sysd: SystemDef, qcart, seed: int = 0, kmesh_subset=None):
    """Everything a Liouvillian needs for a benchmark-shaped system, without an SCF.

    Returns dict(qset, points=[(xk, mill, evc, et, vkb)], vrs, rho, dvan):
    spheres per distinct role vector, smooth random orthonormal occupied
    spinors (``synthetic_ground_state``), Gaussian projector tables, the
    time-reversal-invariant D matrix and smooth fields.  kmesh_subset keeps
    only those mesh points (used for bounded CPU samples).
    """
    if kmesh_subset is not None:
        sysd = SystemDef(name=sysd.name, cell=sysd.cell, atoms=sysd.atoms, ecut=sysd.ecut, fft=sysd.fft,
                         nbnd=sysd.nbnd, kmesh=np.asarray(sysd.kmesh)[list(kmesh_subset)], seed=sysd.seed,
                         notes=sysd.notes)
    qs = qset_exact(sysd, qcart, bitwise=True)
    points = []
    cache = {}
    for i, p in enumerate(qs.points):
        neg = tuple((-p).tolist())
        if neg in cache:  # the negated point: negate its sphere exactly
            mill = -cache[neg]
        else:
            mill = sphere(sysd, p)
        cache[tuple(p.tolist())] = mill
        evc, et = synthetic_ground_state(sysd, p, mill, seed=seed * 100003 + i)
        vkb = projector_table(sysd, p, mill)
        points.append((p, mill, evc, et, vkb))
    vrs, rho = synthetic_fields(sysd, seed)
    return dict(sysd=sysd, qset=qs, points=points, vrs=vrs, rho=rho, dvan=dmatrix(sysd))


def q_path(n: int = 24, q_min: float = 0.02, verts=((0.0, 0.0, 0.0), (0.5, 0.0, 0.0),
                                                     (1.0 / 3.0, 1.0 / 3.0, 0.0), (0.0, 0.0, 0.0))):
    """n fractional q points along the polyline verts (default Gamma -> M(1/2,0,0)
    -> K(1/3,1/3,0) -> Gamma), equally spaced by path length in fractional
    units, the first and last q_min away from the start and end."""
    v = np.asarray(verts, dtype=float)
    seg = np.linalg.norm(np.diff(v, axis=0), axis=1)
    ends = np.cumsum(seg)
    total = ends[-1]
    out = []
    for t in q_min + (total - 2 * q_min) * np.arange(n) / max(n - 1, 1):
        i = int(min(np.searchsorted(ends, t), len(seg) - 1))
        t0 = ends[i] - seg[i]
        out.append(v[i] + (v[i + 1] - v[i]) * (t - t0) / seg[i])
    return np.array(out)


def synthetic_inputs_multi(sysd: SystemDef, qcarts, seed: int = 0):
    """synthetic_inputs for several q sets sharing one point list.

    Returns dict(sysd, xq[nq][3], roles[nq][nk][4], shifts[nq][nk][4][3],
    points=[(xk, mill, evc, et, vkb)], vrs, rho, dvan); every distinct role
    vector (compared bit for bit) is one point, a negated point gets the
    negated sphere of its partner.
    """
    km = kmesh_cart(sysd)
    qcarts = np.asarray(qcarts, dtype=float)
    pts: list = []
    index: dict = {}

    def idx(v):
        key = tuple(np.asarray(v, dtype=float).tolist())
        if key not in index:
            index[key] = len(pts)
            pts.append(np.asarray(v, dtype=float))
        return index[key]

    roles = np.zeros((len(qcarts), len(km), 4), dtype=np.int32)
    for iq, q in enumerate(qcarts):
        for ik, k in enumerate(km):
            roles[iq, ik] = [idx(k), idx(-k), idx(k + q), idx(-k - q)]
    points = []
    cache: dict = {}
    for i, p in enumerate(pts):
        neg = tuple((-p).tolist())
        mill = -cache[neg] if neg in cache else sphere(sysd, p)
        cache[tuple(p.tolist())] = mill
        evc, et = synthetic_ground_state(sysd, p, mill, seed=seed * 100003 + i)
        points.append((p, mill, evc, et, projector_table(sysd, p, mill)))
    vrs, rho = synthetic_fields(sysd, seed)
    return dict(sysd=sysd, xq=qcarts, roles=roles, shifts=np.zeros(roles.shape + (3,), dtype=np.int32),
                points=points, vrs=vrs, rho=rho, dvan=dmatrix(sysd))


def synthetic_fields(sysd: SystemDef, seed: int, bmag: float = 0.1):
    """Smooth synthetic ground-state fields for benchmark shapes.

    Returns (vrs[4], rho[4]) on the grid: vrs = (v_eff, B_x, B_y, B_z) and
    rho = (n, m_x, m_y, m_z).  v_eff is the Gaussian-well local potential;
    n is a sum of atom-centred Gaussians plus a floor, m = 0.3 n along z and
    B = -bmag * n/max(n) along z.
    """
    rng = np.random.default_rng(seed)
    v = vloc_grid(sysd)
    n = _image_sum(sysd, lambda r2, at: 0.05 * np.exp(-r2 / (2 * (1.5 * at.width) ** 2)),
                   images=(1, 1, 1)) + 2e-3
    n *= 1.0 + 0.01 * rng.standard_normal(n.shape)
    m = np.zeros((3,) + n.shape)
    m[2] = 0.3 * n
    b = np.zeros((3,) + n.shape)
    b[2] = -bmag * n / n.max()
    vrs = np.concatenate([v[None], b])
    rho = np.concatenate([n[None], m])
    return vrs, rho
