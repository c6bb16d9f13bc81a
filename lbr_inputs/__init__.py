"""Seeded synthetic inputs shared by the GPU library's tests and the oracle's tests.

This module only draws random numbers and lays out geometry and case
parameters.  It holds none of the lattice-Boltzmann, turbulence-model or
wall-model arithmetic: both the HIP library and the CPU oracle receive the
arrays produced here and do all of the method's work themselves.

The paper's own benchmarks (the TMR NACA 0012 and the MD-30P30N geometries)
are not available, so seeded airfoil-like polylines with the paper's
thickness, Reynolds number, Mach number and angle of attack stand in for them
(Section 3.1.1 and Section 3.2 of the paper).
"""
from __future__ import annotations

import math

import numpy as np

# Boundary-condition codes shared by both configuration structs.
BC_PERIODIC = 0
BC_INLET = 1
BC_OUTLET = 2
BC_SYMMETRY = 3
BC_WALL = 4

WALL_VN = 0
WALL_NISHIMURA = 1
WALL_NOSLIP = 2
WALL_PRESCRIBED = 3

BB_AUTO = 0      # Yu's interpolated scheme at every cut link (step 6 of the VN procedure)
BB_YU = 1        # same as BB_AUTO
BB_HALFWAY = 2   # half-way rule eq (24) at every cut link

BODY_SOLID = 0   # bodies are walls
BODY_REFINE = 1  # bodies only mark where the grid is refined
OUTLET_EXTRAP2 = 0   # outlet populations extrapolated to second order (two upstream cells)
OUTLET_EXTRAP1 = 1   # outlet populations copied from the next upstream cell
OUTLET_PRESSURE = 2  # Zou-He outlet at the reference density

SA_FROZEN = 0
SA_LW = 1
SA_UPWIND1 = 2


def _thickness_coeffs(rng: np.random.Generator):
    """Draw the coefficients of a symmetric thickness polynomial.

    y_t(x) = a0 sqrt(x) + a1 x + a2 x^2 + a3 x^3 + a4 x^4 with a1 chosen so that
    y_t(1) = 0 (sharp trailing edge).  Draws that are negative anywhere on
    (0, 1) are rejected.
    """
    xs = np.linspace(1e-6, 1.0 - 1e-6, 4001)
    while True:
        a0 = rng.uniform(0.26, 0.32)
        a2 = rng.uniform(-0.40, -0.30)
        a3 = rng.uniform(0.20, 0.32)
        a4 = rng.uniform(-0.12, -0.08)
        a1 = -(a0 + a2 + a3 + a4)
        yt = a0 * np.sqrt(xs) + a1 * xs + a2 * xs**2 + a3 * xs**3 + a4 * xs**4
        if np.all(yt > 0.0):
            return np.array([a0, a1, a2, a3, a4])


def _thickness(coef, x):
    a0, a1, a2, a3, a4 = coef
    return a0 * np.sqrt(x) + a1 * x + a2 * x**2 + a3 * x**3 + a4 * x**4


def rotate(xy: np.ndarray, alpha_deg: float, pivot=(0.25, 0.0)) -> np.ndarray:
    """Rotate points by -alpha about the pivot (positive alpha = nose up in a +x stream)."""
    a = -math.radians(alpha_deg)
    c, s = math.cos(a), math.sin(a)
    p = np.asarray(xy, dtype=np.float64) - np.asarray(pivot)
    out = np.empty_like(p)
    out[:, 0] = c * p[:, 0] - s * p[:, 1]
    out[:, 1] = s * p[:, 0] + c * p[:, 1]
    return out + np.asarray(pivot)


def airfoil_polyline(seed: int, n_side: int = 2048, thickness: float = 0.12,
                     alpha_deg: float = 0.0, camber: float = 0.0,
                     camber_pos: float = 0.4) -> np.ndarray:
    """Closed counter-clockwise polyline of a seeded airfoil-like section.

    Unit chord from (0, 0) to (1, 0) before rotation; ``n_side`` points per side
    with cosine spacing, rounded leading edge (sqrt term) and a sharp trailing
    edge.  The first point is the trailing edge; the upper surface runs to the
    leading edge and the lower surface back, so the fluid lies to the right of
    the direction of travel.  The polyline is returned without repeating the
    first point (shape (2 * n_side, 2)).
    """
    rng = np.random.default_rng(seed)
    coef = _thickness_coeffs(rng)
    xs = np.linspace(0.0, 1.0, 20001)
    scale = 0.5 * thickness / _thickness(coef, xs).max()
    j = np.arange(n_side)
    xu = 0.5 * (1.0 + np.cos(np.pi * j / n_side))        # 1 -> ~0
    xl = 0.5 * (1.0 - np.cos(np.pi * j / n_side))        # 0 -> ~1
    ytu = scale * _thickness(coef, xu)
    ytl = scale * _thickness(coef, xl)
    if camber != 0.0:
        def yc(x):
            p = camber_pos
            return np.where(x < p, camber / p**2 * (2 * p * x - x**2),
                            camber / (1 - p)**2 * ((1 - 2 * p) + 2 * p * x - x**2))
        ycu, ycl = yc(xu), yc(xl)
    else:
        ycu = np.zeros_like(xu)
        ycl = np.zeros_like(xl)
    upper = np.stack([xu, ycu + ytu], axis=1)
    lower = np.stack([xl, ycl - ytl], axis=1)
    upper[0, 1] = 0.0 + (ycu[0] if camber != 0.0 else 0.0)   # exact sharp trailing edge
    xy = np.concatenate([upper, lower], axis=0)
    if alpha_deg != 0.0:
        xy = rotate(xy, alpha_deg)
    return np.ascontiguousarray(xy)


def channel_noise(seed: int, nx: int, ny: int):
    """Uniform noise in (-1, 1) for the two velocity components of an nx-by-ny channel."""
    rng = np.random.default_rng(seed)
    xi_x = rng.uniform(-1.0, 1.0, size=(ny, nx))
    xi_y = rng.uniform(-1.0, 1.0, size=(ny, nx))
    return xi_x, xi_y


def random_populations(seed: int, n: int, amplitude: float = 0.02):
    """Random positive D2Q9-like population sets (n, 9) for kernel-level checks."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return w[None, :] * (1.0 + amplitude * rng.uniform(-1, 1, size=(n, 9)))


# ---------------------------------------------------------------------------
# Case definitions (pure data).  Lengths are in chord units; the lattice is
# defined by the level-0 cell size dx0 and the number of refinement levels.
# ---------------------------------------------------------------------------

def case_channel(nx: int = 256, ny: int = 64, steps: int = 2000):
    """Periodic plane channel driven by a body force, walls at halfway links.

    Lattice values for Re_tau = 2000 with a bulk velocity of 0.1 c_s
    (u_tau from the bulk velocity divided by the mean of the wall function over
    the half channel, nu = u_tau h / Re_tau, F = u_tau^2 / h, h = ny / 2).
    """
    return dict(
        name="channel", nx0=nx, ny0=ny, n_levels=1, dx0=1.0, origin=(0.0, 0.0),
        bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL), wall_y=(0.0, float(ny)),
        bands=(), u_ref=0.05773502691896258, nu0=4.372943019927448e-05,
        force=(2.3343054999428939e-07, 0.0), mach=0.1, reynolds=0.0, ref_length=float(ny),
        chi_init=3.0, chi_inlet=3.0, omega_b=1.0, d_wr=2.0, d_wv=1.0,
        wall_model=WALL_VN, bb_mode=BB_AUTO, sa_mode=SA_LW, steps=steps,
        noise_seed=1234, noise_amplitude=1e-3, bodies=[],
    )


def case_airfoil(seed: int = 0, finest_cells_per_chord: int = 1024, n_levels: int = 8,
                 domain_chords: float = 40.0, band_finest: float = 0.25,
                 mach: float = 0.15, reynolds: float = 6e6, alpha_deg: float = 10.0,
                 n_side: int = 2048, thickness: float = 0.12, outlet: int = OUTLET_EXTRAP2,
                 sponge_fraction: float = 0.075, sponge_strength: float = 0.1):
    """Single airfoil-like body in a square domain with distance-band refinement.

    Level l (l = 0 coarsest) has cell size dx0 / 2^l; cells of level l-1 whose
    centre lies within bands[l] of the body are refined, with bands doubling
    towards the coarse levels (band_finest at the finest level).  An absorbing
    layer of sponge_fraction of the level-0 width lines the four far-field sides.
    """
    dx_f = 1.0 / finest_cells_per_chord
    dx0 = dx_f * 2 ** (n_levels - 1)
    n0 = int(round(domain_chords / dx0))
    half = 0.5 * n0 * dx0
    bands = tuple([0.0] + [band_finest * 2 ** (n_levels - 1 - l) for l in range(1, n_levels)])
    xy = airfoil_polyline(seed, n_side=n_side, thickness=thickness, alpha_deg=alpha_deg)
    return dict(
        name="airfoil", nx0=n0, ny0=n0, n_levels=n_levels, dx0=dx0,
        origin=(0.5 - half, -half), bc=(BC_INLET, BC_OUTLET, BC_SYMMETRY, BC_SYMMETRY),
        wall_y=(0.0, 0.0), bands=bands, u_ref=0.0, nu0=0.0, force=(0.0, 0.0),
        mach=mach, reynolds=reynolds, ref_length=1.0, chi_init=3.0, chi_inlet=3.0,
        omega_b=1.0, d_wr=2.0, d_wv=1.0, wall_model=WALL_VN, bb_mode=BB_AUTO,
        sa_mode=SA_LW, alpha_deg=alpha_deg, bodies=[xy], outlet=outlet,
        sponge_width=float(round(sponge_fraction * n0)), sponge_strength=sponge_strength,
    )


def case_airfoil_small(seed: int = 0, alpha_deg: float = 10.0, n_side: int = 256):
    """Down-scaled airfoil case the oracle steps in seconds: 3 levels, finest c/64, 8c domain."""
    return case_airfoil(seed=seed, finest_cells_per_chord=64, n_levels=3, domain_chords=8.0,
                        band_finest=0.25, alpha_deg=alpha_deg, n_side=n_side)


def _min_distance(a: np.ndarray, b: np.ndarray) -> float:
    """Smallest point-to-point distance between two polylines (dense sampling)."""
    d = np.inf
    for k in range(0, len(a), 256):
        blk = a[k:k + 256]
        d = min(d, float(np.sqrt(((blk[:, None, :] - b[None, :, :]) ** 2).sum(-1)).min()))
    return d


def three_element_polylines(seed: int = 0, n_side: int = 1024, alpha_deg: float = 8.0,
                            deflection_deg: float = 30.0, gap: float = 0.02,
                            thickness=(0.16, 0.15, 0.15)):
    """Seeded slat, main element and flap (stand-in for the MD-30P30N of Section 3.2).

    Main element: chord 0.8, seeded camber in [0.02, 0.05].  Slat chord 0.15 and
    flap chord 0.30 (each +-10 %, seeded); thicknesses (slat, main, flap) 16, 15
    and 15 % (blunt leading edges keep the suction peaks within the lattice Mach
    range of D2Q9); both deflected by ``deflection_deg`` (slat nose down about its trailing
    edge, flap trailing edge down about its leading edge) and placed with
    ``gap`` clearance; the assembly is rotated by -alpha about (0.25, 0).  Each
    element is a closed CCW polyline of 2 * n_side points.  The smallest
    distance between elements is at least half the gap.
    """
    rng = np.random.default_rng(1000 + seed)
    camber = rng.uniform(0.02, 0.05)
    cs = 0.15 * rng.uniform(0.9, 1.1)
    cf = 0.30 * rng.uniform(0.9, 1.1)
    ts, tm, tf = thickness
    main = 0.8 * airfoil_polyline(seed, n_side=n_side, thickness=tm, camber=camber)
    slat = cs * airfoil_polyline(seed + 1, n_side=n_side, thickness=ts, camber=0.03)
    flap = cf * airfoil_polyline(seed + 2, n_side=n_side, thickness=tf, camber=0.03)
    # slat: nose down about its trailing edge (cs, 0); flap: trailing edge down about (0, 0)
    slat = rotate(slat, -deflection_deg, pivot=(cs, 0.0))
    flap = rotate(flap, deflection_deg, pivot=(0.0, 0.0))
    # place the slat trailing edge ahead of and above the main leading edge, the flap
    # leading edge below the main trailing edge, then open the gaps until clear
    le_main = main[np.argmin(main[:, 0])]
    te_main = main[0]
    s_off = np.array([le_main[0] - cs + 0.01, le_main[1] + 0.02])
    f_off = np.array([te_main[0] - 0.03, te_main[1] - 0.03])
    for _ in range(200):
        if _min_distance(slat + s_off, main) >= gap:
            break
        s_off += np.array([-0.002, 0.002])
    for _ in range(200):
        if _min_distance(flap + f_off, main) >= gap:
            break
        f_off += np.array([0.002, -0.002])
    bodies = [slat + s_off, main, flap + f_off]
    return [np.ascontiguousarray(rotate(b, alpha_deg)) for b in bodies]


def case_three_element(seed: int = 0, finest_cells_per_chord: int = 4096, n_levels: int = 8,
                       domain_chords: float = 40.0, band_finest: float = 0.165,
                       mach: float = 0.2, reynolds: float = 9e6, alpha_deg: float = 8.0,
                       n_side: int = 1024, thickness=(0.16, 0.15, 0.15)):
    """Three-element high-lift-like configuration: Re 9e6, Mach 0.2, 8 degrees,
    finest c/4096 in a 40-chord domain, 8 levels from c/32 (the distance bands of
    more levels would leave the domain)."""
    case = case_airfoil(seed=seed, finest_cells_per_chord=finest_cells_per_chord,
                        n_levels=n_levels, domain_chords=domain_chords, band_finest=band_finest,
                        mach=mach, reynolds=reynolds, alpha_deg=alpha_deg, n_side=16)
    # the explicit SA diffusion is stable only while (1/sigma) times the sum of the four
    # face diffusivities stays below 1; the eddy viscosity of this case's flap wake on
    # the finest level exceeds that, so its face diffusivities are limited to 0.2 sigma
    case.update(name="three_element", ramp_steps=1000.0, ramp_start=0.25, sa_mu_cap=0.2 * (2.0 / 3.0),
                bodies=three_element_polylines(seed, n_side=n_side, alpha_deg=alpha_deg,
                                               thickness=thickness))
    return case


def _estimate_cells(S: float, D0: float, L: int, finest: int) -> float:
    """Rough fluid-cell count of a single 12 %-thick body in an S x S domain with
    distance bands D0 2^(L-1-l) (Steiner area of each band region)."""
    perim, area = 2.05, 0.08

    def region(D):
        return area + perim * D + np.pi * D * D
    total = 0.0
    for l in range(L):
        dx = 2.0 ** (L - 1 - l) / finest
        outer = S * S if l == 0 else region(D0 * 2 ** (L - 1 - l))
        inner = region(D0 * 2 ** (L - 2 - l)) if l + 1 < L else area
        total += max(outer - inner, 0.0) / (dx * dx)
    return total


def case_sweep(k: int, seed: int = 0, finest_cells_per_chord: int = 512):
    """Case k (0..15) of the batched angle-of-attack sweep: its own seeded body,
    alpha = -4 + 4k/3 degrees, 3 + (k mod 3) levels, finest c/512, and a domain
    width S in [8c, 20c] and finest band D0 in [0.25c, 1c] chosen so that the
    estimated cell count is closest to a seeded target drawn log-uniformly in
    [0.5M, 4M] (the level-1 band must stay clear of the absorbing layer).  The
    case records its estimate and the range of estimates the feasible domains
    and bands span: a target outside that range is met at its nearest end."""
    rng = np.random.default_rng(5000 + seed)
    targets = np.exp(rng.uniform(np.log(0.5e6), np.log(4e6), size=16))
    L = 3 + (k % 3)
    alpha = -4.0 + 4.0 * k / 3.0
    best = None
    lo, hi = np.inf, 0.0
    for S in np.linspace(8.0, 20.0, 49):
        dx0 = 2.0 ** (L - 1) / finest_cells_per_chord
        for D0 in np.linspace(0.25, 1.0, 31):
            band1 = D0 * 2 ** (L - 2)
            if band1 + 0.5 > 0.425 * S - 4 * dx0 * 2:
                continue
            est = _estimate_cells(S, D0, L, finest_cells_per_chord)
            lo, hi = min(lo, est), max(hi, est)
            err = abs(np.log(est / targets[k]))
            if best is None or err < best[0]:
                best = (err, S, D0, est)
    _, S, D0, est = best
    case = case_airfoil(seed=100 + seed * 16 + k, finest_cells_per_chord=finest_cells_per_chord,
                        n_levels=L, domain_chords=float(S), band_finest=float(D0),
                        alpha_deg=alpha, n_side=512)
    case.update(name=f"sweep{k}", target_cells=float(targets[k]), cells_estimate=float(est),
                feasible_cells=(float(lo), float(hi)))
    return case


def case_airfoil_2M(seed: int = 0):
    """The benchmark airfoil: one body, 8 levels from c/8 to c/1024 (about 2.0M cells),
    40-chord domain, Re 6e6, Mach 0.15, 10 degrees."""
    return case_airfoil(seed=seed)


def seeded_level_state(case, level, gx0, gy0, nx, ny, seed, chi_range=(-5.0, 40.0),
                       still_centre=None, still_radius=0.0, wave=0.2):
    """Seeded initial fields over one level's I/O box (cells gx0.. x gy0.., nx x ny):
    rho = 1 + 0.01 xi, a smooth velocity U (1 + a sin(2 pi x / 0.5) cos(2 pi y / 0.5),
    a/2 cos(2 pi x / 0.5) sin(2 pi y / 0.5)) with a = wave, exactly zero within
    still_radius (chord units) of still_centre, and chi uniform in chi_range (xi
    uniform in (-1, 1), numpy PCG64 with the seed and the level).  Returns
    (rho, ux, uy, chi), each (ny, nx)."""
    rng = np.random.default_rng([seed, level])
    dx = case["dx0"] / 2 ** level
    x = case["origin"][0] + (gx0 + np.arange(nx) + 0.5) * dx
    y = case["origin"][1] + (gy0 + np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    U = case["u_ref"] if case["u_ref"] > 0 else case["mach"] / np.sqrt(3.0)
    k = 2.0 * np.pi / 0.5
    ux = U * (1.0 + wave * np.sin(k * X) * np.cos(k * Y))
    uy = 0.5 * wave * U * np.cos(k * X) * np.sin(k * Y)
    if still_centre is not None:
        still = (X - still_centre[0]) ** 2 + (Y - still_centre[1]) ** 2 < still_radius**2
        ux[still] = 0.0
        uy[still] = 0.0
    rho = 1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=(ny, nx))
    chi = rng.uniform(chi_range[0], chi_range[1], size=(ny, nx))
    return rho, np.ascontiguousarray(ux), np.ascontiguousarray(uy), chi


def channel_initial_velocity(case):
    """Laminar profile 1.5 U_b (1 - ((y - h) / h)^2) plus seeded uniform noise on both components.

    Returns (ux, uy), each of shape (ny, nx), at the cell centres y = j + 1/2.
    """
    nx, ny = case["nx0"], case["ny0"]
    h = 0.5 * ny
    ub = case["u_ref"]
    y = np.arange(ny) + 0.5
    prof = 1.5 * ub * (1.0 - ((y - h) / h) ** 2)
    xi_x, xi_y = channel_noise(case["noise_seed"], nx, ny)
    amp = case["noise_amplitude"] * ub
    ux = prof[:, None] + amp * xi_x
    uy = amp * xi_y
    return np.ascontiguousarray(ux), np.ascontiguousarray(uy)


# Precomputed cut-link lists: the record layout of both codes' cut-link input
# (gi, gj, IW x, IW y, normal x, normal y, d_WB, body, q1..q8; q = -1 where a
# link is not cut) and its text file.
CUT_STRIDE = 16
_WALL_COLUMNS = (0, 1, 2, 3, 4, 5, 6, 15) + tuple(range(19, 27))


def cut_link_records(wall: np.ndarray) -> np.ndarray:
    """The cut-link records of a wall-record table (28 columns: gi, gj, IW,
    normal, d_WB, ..., body in column 15, q1..q8 in columns 19-26)."""
    return np.ascontiguousarray(np.asarray(wall, dtype=np.float64)[:, _WALL_COLUMNS])


def perturbed_cut_links(rec: np.ndarray, seed: int, dq: float = 0.15, q_min: float = 0.05,
                        d_iw: float = 0.05, d_angle: float = 0.05, d_dwb: float = 0.05) -> np.ndarray:
    """A seeded stand-in for the output of another preprocessor: every cut link's
    q moved by up to dq (kept in [q_min, 1]), IW by up to d_iw per coordinate,
    the normal turned by up to d_angle radians (still a unit vector) and d_WB
    moved by up to d_dwb (kept >= 0).  Uncut links stay -1."""
    rng = np.random.default_rng(seed)
    r = np.array(rec, dtype=np.float64, copy=True)
    n = len(r)
    q = r[:, 8:16]
    cut = q >= 0
    q[cut] = np.clip(q[cut] + dq * rng.uniform(-1.0, 1.0, int(cut.sum())), q_min, 1.0)
    r[:, 2:4] += d_iw * rng.uniform(-1.0, 1.0, (n, 2))
    a = d_angle * rng.uniform(-1.0, 1.0, n)
    nx, ny = r[:, 4].copy(), r[:, 5].copy()
    r[:, 4] = np.cos(a) * nx - np.sin(a) * ny
    r[:, 5] = np.sin(a) * nx + np.cos(a) * ny
    r[:, 6] = np.maximum(r[:, 6] + d_dwb * rng.uniform(-1.0, 1.0, n), 0.0)
    return r


def write_cut_links(path, lists: dict, comment: str = "") -> None:
    """Writes {level: (n, CUT_STRIDE) records} as a cut-link file ("lbr-cut-links 1",
    then "level l n" blocks; 17 significant digits, so every double round-trips)."""
    with open(path, "w") as fh:
        if comment:
            for line in comment.splitlines():
                fh.write(f"# {line}\n")
        fh.write("lbr-cut-links 1\n")
        for level in sorted(lists):
            rec = np.asarray(lists[level], dtype=np.float64).reshape(-1, CUT_STRIDE)
            fh.write(f"level {int(level)} {len(rec)}\n")
            for row in rec:
                fh.write(" ".join(f"{v:.17g}" for v in row) + "\n")
