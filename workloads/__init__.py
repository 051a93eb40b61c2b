"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path.

This module holds none of the method's arithmetic.  It produces:
  * hexahedral periodic box meshes: geometry node positions on the
    Gauss-Lobatto points of each element (taken from numpy's Legendre
    routines), optional smooth curving, optional random relabelling of each
    element's reference axes, and the face connectivity with orientation codes;
  * initial states sampled from closed forms at given points (manufactured
    solution, Taylor-Green vortex, blast, uniform flow, shear wave);
  * the parameter sets of the benchmark workloads and the served request stream.

Orientation code of a face (used by the HIP library's mesh input): own face
coordinates (p, q) -> neighbour face coordinates: (a, b) = (q, p) if bit0
else (p, q); p' = N - a if bit1 else a; q' = N - b if bit2 else b.  Face
coordinates run along the two other reference axes in increasing order.
Local faces: 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as _leg

# --------------------------------------------------------------------------
# reference points (library routines, used only to place sample points)
# --------------------------------------------------------------------------


def gl_points(N: int) -> np.ndarray:
    """Gauss-Legendre points of degree N (N+1 points), from numpy."""
    return np.polynomial.legendre.leggauss(N + 1)[0]


def lgl_points(N: int) -> np.ndarray:
    """Gauss-Lobatto points of degree N (N+1 points): +-1 and the roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(_leg.Legendre.basis(N).deriv().roots().real)
    pts = np.concatenate([[-1.0], inner, [1.0]])
    # symmetrise exactly so relabelled elements sample identical points
    return 0.5 * (pts - pts[::-1])


def ref_points(N: int, node_type: int) -> np.ndarray:
    return gl_points(N) if node_type == 0 else lgl_points(N)


# --------------------------------------------------------------------------
# proper rotations of the reference cube (signed permutation matrices, det +1)
# --------------------------------------------------------------------------


def _rotations():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            A = np.zeros((3, 3), dtype=int)
            for r in range(3):
                A[r, perm[r]] = signs[r]
            if round(np.linalg.det(A)) == 1:
                mats.append(A)
    return mats


ROTATIONS = _rotations()  # 24 matrices; index 0 is the identity
assert (ROTATIONS[0] == np.eye(3, dtype=int)).all()


def apply_orient(code: int, p, q, N: int):
    a, b = (q, p) if code & 1 else (p, q)
    pp = N - a if code & 2 else a
    qq = N - b if code & 4 else b
    return pp, qq


def _tangential(d):
    return [a for a in range(3) if a != d]


def _face_node_index(f, p, q, N):
    """local (i,j,k) index vector of face node (p,q) on local face f"""
    d = f // 2
    idx = [0, 0, 0]
    idx[d] = N if f % 2 else 0
    t = _tangential(d)
    idx[t[0]] = p
    idx[t[1]] = q
    return idx


def _to_canonical(A, idx, N):
    """index vector in the element's own frame -> canonical (structured) frame"""
    out = [0, 0, 0]
    for r in range(3):
        c = int(np.nonzero(A[r])[0][0])
        out[r] = idx[c] if A[r, c] > 0 else N - idx[c]
    return out


def _local_face_to_canonical(A, f):
    d, s = f // 2, (1 if f % 2 else -1)
    v = np.zeros(3, dtype=int)
    v[d] = s
    vc = A @ v
    dc = int(np.argmax(np.abs(vc)))
    return 2 * dc + (1 if vc[dc] > 0 else 0)


def _canonical_face_to_local(A, fc):
    return _local_face_to_canonical(A.T, fc)


def _build_orient_table():
    """table[rA][f] -> for each rB: (local face of B, code) across a shared canonical face"""
    n = 3  # any grid with >= 2 points fixes the dihedral map
    Nn = n - 1
    table = {}
    for ra, A in enumerate(ROTATIONS):
        for f in range(6):
            fc = _local_face_to_canonical(A, f)
            dc = fc // 2
            tc = _tangential(dc)
            fc2 = fc ^ 1
            for rb, B in enumerate(ROTATIONS):
                f2 = _canonical_face_to_local(B, fc2)
                lookup = {}
                for q in range(n):
                    for p in range(n):
                        ci = _to_canonical(B, _face_node_index(f2, p, q, Nn), Nn)
                        lookup[(ci[tc[0]], ci[tc[1]])] = (p, q)
                mapping = {}
                for q in range(n):
                    for p in range(n):
                        ci = _to_canonical(A, _face_node_index(f, p, q, Nn), Nn)
                        mapping[(p, q)] = lookup[(ci[tc[0]], ci[tc[1]])]
                code = None
                for c in range(8):
                    if all(apply_orient(c, p, q, Nn) == mapping[(p, q)] for (p, q) in mapping):
                        code = c
                        break
                assert code is not None
                table[(ra, f, rb)] = (f2, code)
    return table


_ORIENT_TABLE = None


def _orient_table():
    global _ORIENT_TABLE
    if _ORIENT_TABLE is None:
        _ORIENT_TABLE = _build_orient_table()
    return _ORIENT_TABLE


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------


@dataclass
class Mesh:
    K: tuple
    lo: np.ndarray
    hi: np.ndarray
    ngeo: int
    amp: float
    phases: np.ndarray  # (3,3)
    rot: np.ndarray  # (E,) rotation index per element
    x_geo: np.ndarray  # (E, 3, (ngeo+1)^3) float64, i fastest
    nbr_elem: np.ndarray  # (E, 6) int64
    nbr_face: np.ndarray  # (E, 6) int8
    nbr_orient: np.ndarray  # (E, 6) int8
    period: np.ndarray = field(default=None)

    @property
    def n_elems(self) -> int:
        return int(self.K[0] * self.K[1] * self.K[2])

    def mapping(self, Xc: np.ndarray) -> np.ndarray:
        """physical position of canonical box position(s) Xc (..., 3)"""
        if self.amp == 0.0:
            return Xc.copy()
        L = self.hi - self.lo
        out = Xc.copy()
        for m in range(3):
            prod = np.ones(Xc.shape[:-1])
            for a in range(3):
                prod = prod * np.sin(2.0 * np.pi * (Xc[..., a] - self.lo[a]) / L[a] + self.phases[m, a])
            out[..., m] = Xc[..., m] + self.amp * prod
        return out

    def points(self, r: np.ndarray) -> np.ndarray:
        """physical coordinates (3, E, n^3) of the tensor points r (x) r (x) r
        (r symmetric about 0) of every element, in each element's own frame"""
        n = len(r)
        E = self.n_elems
        Kx, Ky, Kz = self.K
        h = (self.hi - self.lo) / np.array(self.K, dtype=float)
        # local reference coordinates of the tensor points, i fastest
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        loc = np.stack([r[ii.ravel()], r[jj.ravel()], r[kk.ravel()]], axis=-1)  # (n3, 3)
        out = np.empty((3, E, n ** 3))
        e = np.arange(E)
        ex, ey, ez = e % Kx, (e // Kx) % Ky, e // (Kx * Ky)
        origin = self.lo[None, :] + np.stack([ex, ey, ez], axis=-1) * h[None, :]
        for ri, A in enumerate(ROTATIONS):
            sel = np.nonzero(self.rot == ri)[0]
            if len(sel) == 0:
                continue
            can = loc @ A.T.astype(float)  # canonical reference coordinates (n3, 3)
            Xc = origin[sel, None, :] + (can[None, :, :] + 1.0) * 0.5 * h[None, None, :]
            X = self.mapping(Xc)
            out[:, sel, :] = np.moveaxis(X, -1, 0)
        return out


def box_mesh(K, lo, hi, ngeo: int, amp: float = 0.0, seed: int = 0, rotate: bool = False,
             rot_seed: int = 1) -> Mesh:
    """Periodic box of Kx*Ky*Kz hexahedra, element e = ex + Kx*(ey + Ky*ez).

    amp > 0 curves it: x = X + amp * (prod_a sin(2 pi (X_a - lo_a)/L_a + phi_{m a}))_m with
    phases phi ~ U[0, 2 pi)^{3x3} from default_rng(seed); the field is periodic.
    rotate=True relabels each element's reference axes by a random proper
    rotation (default_rng(rot_seed)), which exercises all face orientations."""
    if np.isscalar(K):
        K = (int(K),) * 3
    K = tuple(int(k) for k in K)
    lo = np.asarray(lo, dtype=float) * np.ones(3)
    hi = np.asarray(hi, dtype=float) * np.ones(3)
    E = K[0] * K[1] * K[2]
    phases = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, size=(3, 3))
    if rotate:
        rot = np.random.default_rng(rot_seed).integers(0, 24, size=E)
    else:
        rot = np.zeros(E, dtype=np.int64)
    mesh = Mesh(K=K, lo=lo, hi=hi, ngeo=ngeo, amp=float(amp), phases=phases, rot=rot,
                x_geo=None, nbr_elem=None, nbr_face=None, nbr_orient=None, period=hi - lo)
    xg = mesh.points(lgl_points(ngeo))  # (3, E, ng3)
    mesh.x_geo = np.ascontiguousarray(np.moveaxis(xg, 0, 1))
    # connectivity
    Kx, Ky, Kz = K
    e = np.arange(E)
    ec = np.stack([e % Kx, (e // Kx) % Ky, e // (Kx * Ky)], axis=-1)
    nbr_elem = np.empty((E, 6), dtype=np.int64)
    nbr_face = np.empty((E, 6), dtype=np.int8)
    nbr_orient = np.empty((E, 6), dtype=np.int8)
    if not rotate:
        for f in range(6):
            d, s = f // 2, (1 if f % 2 else -1)
            c2 = ec.copy()
            c2[:, d] = (c2[:, d] + s) % K[d]
            nbr_elem[:, f] = c2[:, 0] + Kx * (c2[:, 1] + Ky * c2[:, 2])
            nbr_face[:, f] = f ^ 1
            nbr_orient[:, f] = 0
    else:
        table = _orient_table()
        for ei in range(E):
            A = ROTATIONS[rot[ei]]
            for f in range(6):
                fc = _local_face_to_canonical(A, f)
                d, s = fc // 2, (1 if fc % 2 else -1)
                c2 = ec[ei].copy()
                c2[d] = (c2[d] + s) % K[d]
                e2 = int(c2[0] + Kx * (c2[1] + Ky * c2[2]))
                f2, code = table[(int(rot[ei]), f, int(rot[e2]))]
                nbr_elem[ei, f] = e2
                nbr_face[ei, f] = f2
                nbr_orient[ei, f] = code
    mesh.nbr_elem, mesh.nbr_face, mesh.nbr_orient = nbr_elem, nbr_face, nbr_orient
    return mesh


# --------------------------------------------------------------------------
# initial states (closed forms sampled at points X: (3, E, n3)); output
# conservative state (5, E, n3)
# --------------------------------------------------------------------------


def _cons(rho, u, v, w, p, gamma):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def mms_state(X, t, gamma):
    """rho = 2 + 0.1 sin(pi (x+y+z-t)), u = v = w = 1, p = rho"""
    rho = 2.0 + 0.1 * np.sin(np.pi * (X[0] + X[1] + X[2] - t))
    one = np.ones_like(rho)
    return _cons(rho, one, one, one, rho, gamma)


def tgv_state(X, Ma, gamma, R=1.0, rho0=1.0, U0=1.0, L=1.0):
    """Taylor-Green vortex, Version II (constant temperature T0 = p0/(rho0 R))"""
    x, y, z = X[0] / L, X[1] / L, X[2] / L
    p0 = rho0 * U0 ** 2 / (gamma * Ma ** 2)
    sx, cx, sy, cy, cz = np.sin(x), np.cos(x), np.sin(y), np.cos(y), np.cos(z)
    u = U0 * sx * cy * cz
    v = -U0 * cx * sy * cz
    w = np.zeros_like(u)
    # cos 2a = cos^2 a - sin^2 a
    p = p0 + rho0 * U0 ** 2 / 16.0 * ((cx * cx - sx * sx) + (cy * cy - sy * sy)) * (1.0 + 2.0 * cz * cz)
    rho = rho0 * p / p0
    return _cons(rho, u, v, w, p, gamma)


def blast_state(X, center, period, gamma, radius=0.1, p_in=1000.0, p_out=1.0):
    """rho = 1, u = 0, p = p_in inside the periodic-distance ball, p_out outside"""
    d2 = np.zeros(X.shape[1:])
    for c in range(3):
        dd = X[c] - center[c]
        dd = dd - period[c] * np.round(dd / period[c])
        d2 = d2 + dd * dd
    p = np.where(np.sqrt(d2) < radius, p_in, p_out)
    rho = np.ones_like(p)
    z = np.zeros_like(p)
    return _cons(rho, z, z, z, p, gamma)


def uniform_state(X, rho, vel, p, gamma):
    one = np.ones(X.shape[1:])
    return _cons(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, p * one, gamma)


def shear_wave_state(X, A, k, rho, p, gamma):
    """u = (0, A sin(k x), 0), uniform rho and p"""
    z = np.zeros(X.shape[1:])
    return _cons(rho + z, z, A * np.sin(k * X[0]), z, p + z, gamma)


def random_smooth_state(X, seed, gamma, period):
    """a smooth periodic state with O(1) variation in every variable"""
    g = np.random.default_rng(seed)
    ph = g.uniform(0, 2 * np.pi, size=(5, 3))
    kk = 2 * np.pi / period
    f = [np.sin(kk[0] * X[0] + ph[m, 0]) * np.cos(kk[1] * X[1] + ph[m, 1]) *
         np.sin(kk[2] * X[2] + ph[m, 2]) for m in range(5)]
    rho = 1.0 + 0.3 * f[0]
    u, v, w = 0.4 * f[1], 0.3 * f[2], 0.2 * f[3]
    p = 1.0 + 0.3 * f[4]
    return _cons(rho, u, v, w, p, gamma)


# --------------------------------------------------------------------------
# parameter sets
# --------------------------------------------------------------------------


def params(N, node_type=0, riemann=0, viscous=1, source=0, shock=0, gamma=1.4, R=1.0, Pr=0.72,
           mu=1e-3, precision=0, alpha_max=1.0, alpha_min=0.001, ind_a=0.5, ind_c=1.8,
           ind_s=math.log(9999.0), check_finite=0, alpha_smooth=0, volume_flux=0, viscosity=0,
           T_ref=1.0, time_scheme=0, p_ref=0.0):
    """volume_flux: 0 standard weak form, 1 split form with Pirozzoli's two-point
    flux (Gauss-Lobatto nodes); viscosity: 0 constant mu, 1 Sutherland's law with
    mu = mu(T_ref); time_scheme: 0 five-stage, 1 fourteen-stage low-storage RK;
    p_ref: background pressure the mixed form subtracts in its FP32 fluxes"""
    return dict(N=N, nodes=node_type, riemann=riemann, viscous=viscous, source=source,
                shock_capturing=shock, gamma=gamma, R=R, Pr=Pr, mu=mu, precision=precision,
                alpha_max=alpha_max, alpha_min=alpha_min, ind_a=ind_a, ind_c=ind_c, ind_s=ind_s,
                check_finite=check_finite, alpha_smooth=alpha_smooth, volume_flux=volume_flux,
                viscosity=viscosity, T_ref=T_ref, time_scheme=time_scheme, p_ref=p_ref)


@dataclass
class Workload:
    name: str
    params: dict
    mesh: Mesh
    U0: np.ndarray  # (5, E, n3)
    steps: int
    cfl: float = 0.9
    extra: dict = field(default_factory=dict)

    @property
    def dof(self) -> int:
        return self.mesh.n_elems * (self.params["N"] + 1) ** 3


def mms_workload(K=4, N=3, steps=10, rotate=False):
    """[-1,1]^3 periodic, K^3 Cartesian elements, GL nodes, manufactured solution"""
    mesh = box_mesh(K, -1.0, 1.0, N, rotate=rotate)
    p = params(N, node_type=0, riemann=0, viscous=1, source=1, mu=1e-3)
    X = mesh.points(gl_points(N))
    return Workload("mms", p, mesh, mms_state(X, 0.0, p["gamma"]), steps)


def tgv_workload(K=24, N=7, steps=100, Ma=0.1, Re=1600.0, curved=True, seed=0, precision=0,
                 rotate=False, riemann=1, p_ref=None, ngeo=None):
    """[0,2pi]^3, K^3 elements, GL nodes, Taylor-Green vortex Version II.  The
    mixed form (precision 1) takes the background pressure p0 out of its FP32
    arithmetic unless p_ref says otherwise"""
    mesh = box_mesh(K, 0.0, 2 * np.pi, N if ngeo is None else ngeo, amp=0.05 if curved else 0.0, seed=seed,
                    rotate=rotate)
    if p_ref is None:
        p_ref = 1.0 / (1.4 * Ma * Ma) if precision == 1 else 0.0
    p = params(N, node_type=0, riemann=riemann, viscous=1, source=0, mu=1.0 / Re, precision=precision,
               p_ref=p_ref)
    X = mesh.points(gl_points(N))
    return Workload("tgv", p, mesh, tgv_state(X, Ma, p["gamma"]), steps, extra=dict(Ma=Ma, Re=Re))


def compressible_tgv_workload(K=16, N=7, steps=100, Ma=1.25, Re=1600.0, curved=False, seed=0,
                              rotate=False, alpha_max=1.0, ngeo=None):
    """the supersonic Taylor-Green vortex: [0,2pi]^3, K^3 elements, Gauss-Lobatto
    nodes, Version II at Ma = 1.25, Re = 1600, Sutherland's law with T_ref = T0 and
    Pr = 0.71, split form with Pirozzoli's flux, LLF surface flux, BR1, the modal
    indicator with FV-subcell blending, and the fourteen-stage RK scheme"""
    mesh = box_mesh(K, 0.0, 2 * np.pi, N if ngeo is None else ngeo, amp=0.05 if curved else 0.0, seed=seed,
                    rotate=rotate)
    gamma, R = 1.4, 1.0
    p0 = 1.0 / (gamma * Ma ** 2)
    p = params(N, node_type=1, riemann=0, viscous=1, source=0, shock=1, gamma=gamma, R=R, Pr=0.71,
               mu=1.0 / Re, alpha_max=alpha_max, volume_flux=1, viscosity=1, T_ref=p0 / R,
               time_scheme=1)
    X = mesh.points(lgl_points(N))
    # the fourteen-stage scheme is stable at about 3.2 times the five-stage step
    return Workload("ctgv", p, mesh, tgv_state(X, Ma, gamma, R=R), steps, cfl=2.5,
                    extra=dict(Ma=Ma, Re=Re, p0=p0))


def blast_workload(K=32, N=5, steps=200, seed=0, rotate=False, alpha_smooth=0, viscous=0, ind_a=0.05, cfl=0.9):
    """[-1,1]^3 periodic, K^3 Cartesian elements, LGL nodes, pressure-ratio-1000
    blast, Euler, element-local blending factor with the indicator threshold
    at a tenth of Hennemann's (ind_a = 0.05), CFL 0.9 at t = 0.  With the
    default threshold the element holding the front keeps alpha ~ 0.67 and its
    pressure undershoots below zero; with viscosity the (unblended) DG heat
    flux of the 1000:1 temperature step drives the pressure next to the ball
    negative within a few steps at any alpha."""
    mesh = box_mesh(K, -1.0, 1.0, N, rotate=rotate)
    p = params(N, node_type=1, riemann=0, viscous=viscous, source=0, shock=1, mu=1e-3 if viscous else 0.0,
               alpha_smooth=alpha_smooth, ind_a=ind_a)
    center = np.random.default_rng(seed).uniform(-1.0, 1.0, size=3)
    X = mesh.points(lgl_points(N))
    return Workload("blast", p, mesh, blast_state(X, center, mesh.period, p["gamma"]), steps, cfl=cfl,
                    extra=dict(center=center))


def serving_requests(n=512, seed=0, rate=1.0):
    """the served request stream: drawn per request in this order: inter-arrival
    ~ Exp(rate), K ~ U{4..16}, N ~ U{3,5,7}, Ma ~ U[0.05,0.3], Re ~ U[400,1600],
    steps ~ U{50..400}"""
    g = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n):
        t += g.exponential(1.0 / rate)
        K = int(g.integers(4, 17))
        N = int(g.choice([3, 5, 7]))
        Ma = float(g.uniform(0.05, 0.3))
        Re = float(g.uniform(400.0, 1600.0))
        steps = int(g.integers(50, 401))
        reqs.append(dict(id=i, t_arrival=t, K=K, N=N, Ma=Ma, Re=Re, steps=steps))
    return reqs


_REQUEST_MESHES = {}


def request_workload(req, precision=0):
    """one served request: Cartesian periodic [0,2pi]^3 TGV Version II, Roe, BR1
    (requests of one (K, N) share the mesh object)"""
    N, K = req["N"], req["K"]
    if (K, N) not in _REQUEST_MESHES:
        m = box_mesh(K, 0.0, 2 * np.pi, N)
        _REQUEST_MESHES[(K, N)] = (m, m.points(gl_points(N)))
    mesh, X = _REQUEST_MESHES[(K, N)]
    p = params(N, node_type=0, riemann=1, viscous=1, mu=1.0 / req["Re"], precision=precision,
               p_ref=1.0 / (1.4 * req["Ma"] ** 2) if precision == 1 else 0.0)
    return Workload("tgv_req", p, mesh, tgv_state(X, req["Ma"], p["gamma"]), req["steps"],
                    extra=dict(Ma=req["Ma"], Re=req["Re"]))
