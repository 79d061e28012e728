"""Seeded synthetic workloads: system constants and initial conditions.

This module is the only code shared by the HIP path and the CPU oracle.  It
builds the *inputs* of an integration (physical constants in atomic units and
the 12-component initial states) and holds none of the integrator's or the
force's arithmetic.

State layout (paper Sec. 2.1, definition of y): components 0-2 are the ion's
Cartesian coordinates, 3-5 the ion's velocity, 6-8 the atom's coordinates and
9-11 the atom's velocity.  Ensembles are returned as a float64 array of shape
(12, n): twelve planes of n trajectories, plane c holding component c.

The trap term follows the paper's Hamiltonian (Sec. 2.1): the ion's
acceleration along axis k contains -(a_k + 2 q_k cos(Omega t)) Omega^2/4 x_k.
A trap written as x'' + (Omega^2/4)(a - 2 q cos(Omega t)) x = 0 with
(a, a, -2a) and (q, q, -2q) on (x, y, z) is the same equation with the
paper-form q taken as (-q, -q, +2q); ``paul_trap`` does that conversion.

Initial-condition recipe for the thermal, impact-parameter ensembles
(``thermal_ensemble``), per trajectory i, from one PCG64 stream:
  * 12 uniforms u[i, 0:12] = (raw64 >> 11) * 2**-53 (numpy ``Generator.random``),
    drawn row by row, so trajectory i depends only on the seed and i;
  * five Box-Muller pairs from (u0,u1) ... (u8,u9) give 10 normals, of which the
    first 9 are the ion position, the ion velocity and the atom velocity (3 each);
  * u10 gives the impact parameter b = b_max sqrt(u10), u11 the azimuth
    psi = 2 pi u11 around the atom's direction of flight;
  * ion position ~ N(0, kT_ion / (m_ion w^2)) per axis with the secular frequency
    of the x axis, w = (Omega/2) sqrt(a_x + q_x^2 / 2) (paper Sec. 4.1);
    ion velocity ~ N(0, kT_ion / m_ion); atom velocity ~ N(0, kT_atom / m_atom);
  * the atom starts on the sphere of radius R0 centred on the ion's initial
    position, on the straight line along its own velocity that passes the ion at
    distance b: x_atom = x_ion - sqrt(R0^2 - b^2) v_hat + b (cos psi e1 + sin psi e2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 values used to express SI inputs in atomic units.
AMU = 1822.888486209            # unified atomic mass unit in electron masses
KB = 3.166811563e-6             # Boltzmann constant in Hartree per kelvin
T_AU = 2.4188843265857e-17      # atomic unit of time in seconds

NSTATE = 12

# Observable planes written by both integrators (one float64 plane each).
OBS_NAMES = (
    "tend", "status", "nsteps", "nfailed", "bounces", "lifetime", "angle",
    "transfer", "position", "dist", "ke", "rmin", "hnext",
)
NOBS = len(OBS_NAMES)
OBS = {name: i for i, name in enumerate(OBS_NAMES)}

STATUS_NAMES = {0: "running", 1: "escaped", 2: "tmax", 3: "maxsteps", 4: "hmin", 5: "nonfinite"}
ST_ESCAPED, ST_TMAX, ST_MAXSTEPS, ST_HMIN, ST_NONFINITE = 1, 2, 3, 4, 5


@dataclasses.dataclass
class System:
    """Constants of one atom + trapped-ion system, atomic units (paper Sec. 2.1).

    V(r) = -Cn / r^n + Cm / r^m; trap acceleration on the ion along axis k is
    -(a_k + 2 q_k cos(omega_rf t)) omega_rf^2 / 4 x_k.  ``r_exit`` ends a
    trajectory once the atom-ion distance exceeds it after the first closest
    approach (0 disables that exit), ``r_bounce`` is the distance below which an
    inner turning point counts as a short-range collision ("bounce"),
    ``max_steps`` caps accepted steps and ``hmax`` the step size (0 means one
    tenth of the integration span).
    """

    m_ion: float
    m_atom: float
    n: int = 4
    m: int = 8
    Cn: float = 0.0
    Cm: float = 0.0
    a: tuple = (0.0, 0.0, 0.0)
    q: tuple = (0.0, 0.0, 0.0)
    omega_rf: float = 0.0
    r_exit: float = 0.0
    r_bounce: float = 20.0
    max_steps: int = 1_000_000
    hmax: float = 0.0

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Workload:
    """A complete integration request: system, ensemble recipe and tolerances."""

    name: str
    system: System
    n: int
    seed: int
    t0: float
    tmax: float
    rtol: float
    atol: float
    T_ion: float
    T_atom: float
    R0: float
    b_max: float

    def initial_states(self, n: int | None = None) -> np.ndarray:
        """The (12, n) float64 SoA initial states of this workload's ensemble."""
        return thermal_ensemble(self.system, self.n if n is None else n, self.seed,
                                self.T_ion, self.T_atom, self.R0, self.b_max)


def rf_omega(freq_hz: float) -> float:
    """Angular radio frequency 2 pi f in inverse atomic time units."""
    return 2.0 * math.pi * freq_hz * T_AU


def paul_trap(a: float, q: float) -> tuple[tuple, tuple]:
    """Paper-form (a_k, q_k) for the trap x'' + (Omega^2/4)(a - 2q cos Omega t) x = 0
    on x and y with a_z = -2a, q_z = -2q."""
    return (a, a, -2.0 * a), (-q, -q, 2.0 * q)


def secular_omega_x(system: System) -> float:
    """Secular frequency of the x axis, (Omega/2) sqrt(a_x + q_x^2/2) (paper Sec. 4.1)."""
    return 0.5 * system.omega_rf * math.sqrt(system.a[0] + 0.5 * system.q[0] ** 2)


def liyb_system(q: float = 0.1, a: float = 0.0, r_exit: float = 1e5) -> System:
    """6-amu atom and 171-amu ion, C4 = 82, C8 = 4.1e5 (minimum at r = 10 a0), in a
    2 MHz Paul trap; bounce radius 2 R_e = 20 a0."""
    ta, tq = paul_trap(a, q)
    return System(m_ion=171.0 * AMU, m_atom=6.0 * AMU, n=4, m=8, Cn=82.0, Cm=4.1e5,
                  a=ta, q=tq, omega_rf=rf_omega(2.0e6), r_exit=r_exit, r_bounce=20.0,
                  max_steps=1_000_000, hmax=0.0)


def rf_periods(system: System, k: float) -> float:
    return k * 2.0 * math.pi / system.omega_rf


def thermal_workload(n: int, seed: int = 0, rtol: float = 1e-8, atol: float = 1e-10,
                     T_atom: float = 1e-3, q: float = 0.1, name: str | None = None) -> Workload:
    """Thermal ion (0.5 mK) + Maxwell-Boltzmann atom aimed with impact parameter
    b = b_max sqrt(U) from a sphere of R0 = 1e5 a0 (b_max = 2e4 a0); exit at r > R0
    after closest approach or after 200 RF periods."""
    system = liyb_system(q=q)
    return Workload(name=name or f"thermal-liyb-n{n}", system=system, n=n, seed=seed,
                    t0=0.0, tmax=rf_periods(system, 200.0), rtol=rtol, atol=atol,
                    T_ion=0.5e-3, T_atom=T_atom, R0=1e5, b_max=2e4)


def small_ensemble() -> Workload:
    """1,024 trajectories, seed 0, RelTol 1e-8, AbsTol 1e-10."""
    return thermal_workload(1024, 0, name="liyb-thermal-1k")


def full_ensemble() -> Workload:
    """2^20 trajectories, seed 0, RelTol 1e-8, AbsTol 1e-10."""
    return thermal_workload(1 << 20, 0, name="liyb-thermal-1M")


def cold_collision_workload(n: int, seed: int = 11) -> Workload:
    """An ensemble that forms many complexes, for distribution tests: a 10 uK
    atom aimed with b_max = 1,500 a0 (a few Langevin radii) from R0 = 2e4 a0
    at an ion cooled to 0.1 uK, otherwise the 1,024-trajectory configuration's
    system and tolerances.  About 5.5% of the trajectories form a complex
    (two or more bounces; 906 of 16,384 for seed 11), mostly of two or three
    bounces with lifetimes below a few RF periods."""
    wl = thermal_workload(n, seed, T_atom=1e-5, name=f"cold-collisions-n{n}")
    system = dataclasses.replace(wl.system, r_exit=2e4)
    return dataclasses.replace(wl, system=system, R0=2e4, b_max=1500.0, T_ion=1e-7)


# The batched grid: collision (atom) temperatures log-spaced over 10 uK .. 10 mK
# and Paul-trap q values (a = 0); ensemble sizes log-uniform in [1024, 262144].
BATCH_T_ATOM = tuple(float(t) for t in np.logspace(-5.0, -2.0, 8))
BATCH_Q = (0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7)
BATCH_SIZE_SEED = 1
BATCH_IC_SEED0 = 100


def batch_grid(scale: float = 1.0) -> list[Workload]:
    """The 64 ensembles of the batched configuration, T_atom-major (ensemble
    k = 8 iT + iq).  Size of ensemble k: floor(1024 * 256**U_k) with U_k the
    k-th uniform of a PCG64 stream of seed 1 (``scale`` shrinks every size, at
    least 1, for tests); initial states of ensemble k come from seed 100 + k.
    Everything else is the 1,024-trajectory configuration's: masses,
    potential, 0.5 mK ion, R0, b_max, 200 RF periods, RelTol 1e-8, AbsTol 1e-10.
    For q >= 0.5 the ion's z motion is Mathieu-unstable (|tr M_z| > 2)."""
    u = np.random.Generator(np.random.PCG64(BATCH_SIZE_SEED)).random(len(BATCH_T_ATOM) * len(BATCH_Q))
    out = []
    for it, T in enumerate(BATCH_T_ATOM):
        for iq, q in enumerate(BATCH_Q):
            k = it * len(BATCH_Q) + iq
            n = int(math.floor(1024.0 * 256.0 ** u[k]))
            n = max(1, int(n * scale))
            out.append(thermal_workload(n, BATCH_IC_SEED0 + k, T_atom=T, q=q,
                                        name=f"batch-T{T:.2e}-q{q:g}"))
    return out


# The serving stream: Poisson arrivals at 200 requests/s, sizes floor(256 *
# 4096**U), RelTol from {1e-6, 1e-8, 1e-10} with AbsTol = RelTol / 100, a
# quarter of the requests with single-precision stages, collision temperature
# and trap q drawn from the batched grid's values; each request integrates a
# slice of one pool of initial states, moved to its temperature and q by
# ``retarget_thermal``.
SERVING_SEED = 2
SERVING_RATE_HZ = 200.0
SERVING_RTOLS = (1e-6, 1e-8, 1e-10)
SERVING_POOL = 1 << 21
SERVING_POOL_SEED = 3


@dataclasses.dataclass(frozen=True)
class ServingRequest:
    arrival_s: float      # seconds after the stream starts
    n: int                # trajectories
    offset: int           # first trajectory of its slice of the pool
    rtol: float
    atol: float
    precision: str        # "fp64" or "fp32-stages"
    T_atom: float = 1e-3  # collision (atom) temperature, K
    q: float = 0.1        # Paul-trap q (a = 0)


def serving_stream(count: int, seed: int = SERVING_SEED, rate_hz: float = SERVING_RATE_HZ,
                   max_size: int = 256 * 4096) -> list[ServingRequest]:
    """The first `count` requests of the serving stream.  From one PCG64
    stream of `seed`, per request: an exponential gap (mean 1 / rate_hz), U for
    the size, one uniform each for the tolerance, the precision, the slice
    offset, the temperature and q (each uniform over the batched grid's
    BATCH_T_ATOM and BATCH_Q).  Sizes are capped at max_size (the stream's own
    maximum by default, smaller for tests)."""
    u = np.random.Generator(np.random.PCG64(seed)).random((count, 7))
    t = np.cumsum(-np.log1p(-u[:, 0]) / rate_hz)
    out = []
    for k in range(count):
        n = min(int(math.floor(256.0 * 4096.0 ** u[k, 1])), max_size)
        rtol = SERVING_RTOLS[min(int(u[k, 2] * len(SERVING_RTOLS)), len(SERVING_RTOLS) - 1)]
        precision = "fp32-stages" if u[k, 3] < 0.25 else "fp64"
        offset = int(u[k, 4] * (SERVING_POOL - n + 1))
        T = BATCH_T_ATOM[min(int(u[k, 5] * len(BATCH_T_ATOM)), len(BATCH_T_ATOM) - 1)]
        q = BATCH_Q[min(int(u[k, 6] * len(BATCH_Q)), len(BATCH_Q) - 1)]
        out.append(ServingRequest(float(t[k]), n, offset, rtol, rtol * 1e-2, precision, T, q))
    return out


def serving_pool(n: int = SERVING_POOL) -> Workload:
    """The pool the serving stream's requests slice: the 1,024-trajectory
    configuration's physics (1 mK, q = 0.1, 200 RF periods), seed 3."""
    return thermal_workload(n, SERVING_POOL_SEED, name=f"serving-pool-{n}")


def serving_request_workload(r: ServingRequest) -> Workload:
    """The system, span and recipe of one serving request (its q and
    temperature; the pool's seed and sizes)."""
    wl = thermal_workload(r.n, SERVING_POOL_SEED, rtol=r.rtol, atol=r.atol, T_atom=r.T_atom,
                          q=r.q, name=f"serving-T{r.T_atom:.2e}-q{r.q:g}-n{r.n}")
    return wl


def retarget_thermal(y0, system_from: System, T_atom_from: float, system_to: System,
                     T_atom_to: float):
    """Initial states of ``thermal_ensemble`` drawn for (system_from,
    T_atom_from) moved to (system_to, T_atom_to) with the same uniforms: the
    ion's thermal position scales with 1 / (secular frequency), the atom's
    velocity with sqrt(T_atom), and the atom keeps its offset from the ion
    (the direction of flight, impact parameter and azimuth do not depend on
    either).  Equals the ensemble drawn directly for the new parameters up to
    rounding.  Works on numpy arrays and torch tensors of shape (12, n);
    returns a new array."""
    sx = secular_omega_x(system_from) / secular_omega_x(system_to)
    sv = math.sqrt(T_atom_to / T_atom_from)
    out = y0 * 1.0
    out[0:3] = y0[0:3] * sx
    out[6:9] = y0[6:9] + (out[0:3] - y0[0:3])
    out[9:12] = y0[9:12] * sv
    return out


def _uniform_rows(n: int, seed: int, ncols: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n, ncols))


def _box_muller(u1: np.ndarray, u2: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    rad = np.sqrt(-2.0 * np.log1p(-u1))      # 1 - u1 lies in (0, 1]
    ang = 2.0 * math.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def _perpendicular_basis(vhat: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Two unit vectors completing vhat (rows) to a right-handed orthonormal frame."""
    ref = np.zeros_like(vhat)
    use_x = np.abs(vhat[:, 2]) > 0.9
    ref[~use_x, 2] = 1.0
    ref[use_x, 0] = 1.0
    e1 = np.cross(vhat, ref)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(vhat, e1)
    return e1, e2


def thermal_ensemble(system: System, n: int, seed: int, T_ion: float, T_atom: float,
                     R0: float, b_max: float) -> np.ndarray:
    """(12, n) float64 initial states; the recipe is in the module docstring."""
    if n < 0:
        raise ValueError("n must be >= 0")
    if b_max > R0:
        raise ValueError("b_max must not exceed R0")
    u = _uniform_rows(n, seed, 12)
    normals = np.empty((n, 10))
    for p in range(5):
        z0, z1 = _box_muller(u[:, 2 * p], u[:, 2 * p + 1])
        normals[:, 2 * p] = z0
        normals[:, 2 * p + 1] = z1
    w = secular_omega_x(system)
    sx = math.sqrt(KB * T_ion / system.m_ion) / w if w > 0 else 0.0
    svi = math.sqrt(KB * T_ion / system.m_ion)
    sva = math.sqrt(KB * T_atom / system.m_atom)
    xi = normals[:, 0:3] * sx
    vi = normals[:, 3:6] * svi
    va = normals[:, 6:9] * sva
    b = b_max * np.sqrt(u[:, 10])
    psi = 2.0 * math.pi * u[:, 11]
    speed = np.linalg.norm(va, axis=1, keepdims=True)
    vhat = va / np.where(speed > 0, speed, 1.0)
    vhat[speed[:, 0] == 0] = (0.0, 0.0, 1.0)
    e1, e2 = _perpendicular_basis(vhat)
    along = np.sqrt(R0 * R0 - b * b)[:, None]
    xa = xi - along * vhat + b[:, None] * (np.cos(psi)[:, None] * e1 + np.sin(psi)[:, None] * e2)
    y0 = np.empty((NSTATE, n))
    y0[0:3] = xi.T
    y0[3:6] = vi.T
    y0[6:9] = xa.T
    y0[9:12] = va.T
    return y0


def potential_cn_de(n: int, m: int, Cn: float, De: float) -> float:
    """Cm of V(r) = -Cn/r^n + Cm/r^m from Cn and the well depth De (the
    paper's "CnDe" parameterization, Sec. 4): at the minimum r_e, V'(r_e) = 0
    gives r_e^(m-n) = m Cm / (n Cn) and V(r_e) = -Cn r_e^-n (1 - n/m) = -De."""
    r_e = (Cn * (1.0 - n / m) / De) ** (1.0 / n)
    return n * Cn * r_e ** (m - n) / m


def potential_de_re(n: int, m: int, De: float, Re: float) -> tuple[float, float]:
    """(Cn, Cm) from the well depth De and its position Re (the paper's
    "DeRe" parameterization, Sec. 4)."""
    cn = De * Re**n / (1.0 - n / m)
    return cn, n * cn * Re ** (m - n) / m


def nangles_auto(count: int) -> tuple[int, int]:
    """(n_theta, n_phi) near sqrt(count) with n_theta * n_phi >= count (the
    product may exceed count a little, as in the paper's automatic choice)."""
    nt = max(1, int(math.ceil(math.sqrt(count))))
    return nt, max(1, int(math.ceil(count / nt)))


def angle_grid(n_theta: int, n_phi: int, mode: str = "uniform", theta_min: float = 0.0,
               theta_max: float = math.pi / 2, phi_min: float = 0.0, phi_max: float = math.pi / 2,
               seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Launch directions (theta, phi), n_theta * n_phi of them (the paper's
    "uniform" and "random" positions, Sec. 4).  theta = arccos(1 - 2u) with u
    between (1 - cos theta_min)/2 and (1 - cos theta_max)/2, so equal steps of u
    are equal solid angles.  uniform: n_theta evenly spaced u times n_phi evenly
    spaced phi, every pair (theta-major); random: u and phi uniform from a PCG64
    stream of `seed`.  The default range is the first octant."""
    u_lo, u_hi = (1.0 - math.cos(theta_min)) / 2.0, (1.0 - math.cos(theta_max)) / 2.0
    if mode == "uniform":
        u = np.linspace(u_lo, u_hi, n_theta)
        ph = np.linspace(phi_min, phi_max, n_phi)
        uu, pp = np.meshgrid(u, ph, indexing="ij")
        return np.arccos(1.0 - 2.0 * uu.ravel()), pp.ravel()
    if mode == "random":
        r = np.random.Generator(np.random.PCG64(seed)).random((n_theta * n_phi, 2))
        u = u_lo + (u_hi - u_lo) * r[:, 0]
        return np.arccos(1.0 - 2.0 * u), phi_min + (phi_max - phi_min) * r[:, 1]
    raise ValueError(f"unknown mode {mode!r}")


def head_on_ensemble(system: System, r0: float, T_atom: float, theta: np.ndarray,
                     phi: np.ndarray) -> np.ndarray:
    """(12, N) head-on initial states, one per direction (theta[i], phi[i])."""
    return np.stack([head_on_state(system, r0, T_atom, t, p) for t, p in zip(theta, phi)], axis=1)


def head_on_state(system: System, r0: float, T_atom: float, theta: float, phi: float) -> np.ndarray:
    """Ion at rest at the origin, atom at r0 (sin t cos p, sin t sin p, cos t) moving
    towards it with speed sqrt(3 kT / m_atom) (paper Sec. 2.1, initial conditions)."""
    v0 = math.sqrt(3.0 * KB * T_atom / system.m_atom)
    u = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    y = np.zeros(NSTATE)
    y[6:9] = r0 * u
    y[9:12] = -v0 * u
    return y
