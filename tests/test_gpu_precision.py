"""Storage precision and field parity against the FP64 oracle at a converged
state (needs an MI355X), on the single airfoil and on the three-element case.

The 3-level airfoil (finest c/64, Re 6e6, M 0.15, 10 degrees) is run for 4000
coarse steps, by which the oracle's force coefficients are steady to six
digits.

Fields (FP64 and FP32 storage): every owned cell of every level and every wall
node against the oracle.  FP64: u within 1e-10 U, chi within 1e-10 of
max(|chi|, 1), rho within 1e-12, as in the short windows.  FP32: u within
1e-5 U and rho within 1e-6 (measured 3.4e-6 U and 1e-7), chi within 1e-4 of
the level's largest chi (measured 1.7e-5 to 3.6e-5).  The converged chi
carries what the SA sources added along the streamlines over the whole run:
about half of its FP32 difference comes from the hardware reciprocal and the
exp2 / log2 sixth root of the FP32 SA update (with IEEE division and powf the
same run gives 4e-6 to 1.6e-5, but the step is 10 % slower), the rest from the
rounding of the velocity that enters the vorticity and the convection.

Surface data, every storage (populations in FP64, FP32, FP16, BF16 and mixed
(FP32 on the two finest levels, FP16 below), the 16-bit formats also with the
free-stream shift; FP32 arithmetic, FP64 Newton and force sums):
  * FP64: rounding-order differences only, 1e-9 relative;
  * FP32: the converged-state bounds of the study's measurement plan: Cp
    max-abs 1e-3, Cf max-abs 1 % of max |Cf|, C_D and C_L 1e-3 relative (measured
    5.2e-6, 9.8e-7, 2.3e-7, 8.8e-7);
  * the 16-bit formats: their errors are reported; the formats that the
    equal-Cf comparison counts as meeting the FP32 Cf bound (FP16 and mixed, each
    with the free-stream shift) are asserted to meet it, the others only to stay
    finite.
"""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle
from tests import parity_util as U

pytestmark = pytest.mark.gpu

STEPS = 4000
CF_BOUND = 0.01          # max |dCf| <= 1 % of max |Cf|, the FP32 bound of the comparison
BOUNDS = {  # storage: (Cp max-abs, Cf max-abs / max|Cf|, C_D and C_L relative)
    "f64": (1e-9, 1e-9, 1e-9),
    "f32": (1e-3, CF_BOUND, 1e-3),
}
MEETS_CF_BOUND = ("f16s", "mixeds")


@pytest.fixture(scope="module")
def converged_oracle():
    case = LI.case_airfoil_small()
    o = oracle.Sim(case)
    o.advance(STEPS)
    cp, cf = o.surface(0)
    return case, cp, cf, o.forces(), o


@pytest.mark.parametrize("storage,tol,chi_tol,rho_tol", [("f64", 1e-10, 1e-10, 1e-12), ("f32", 1e-5, 1e-4, 1e-6)])
def test_converged_fields_element_by_element(converged_oracle, storage, tol, chi_tol, rho_tol):
    """The converged state itself, cell by cell on every level and node by node at
    the wall, not only its surface data."""
    case, _, _, _, o = converged_oracle
    g = U.gpu_solver(case, storage)
    g.use_graph(True)
    g.advance(STEPS)
    errs = U.level_errors(g, o, case["n_levels"], U.reference_speed(case))
    print(storage, errs)
    chi_key = "chi" if storage == "f64" else "chi_level"
    for l, e in errs.items():
        assert e["ux"] <= tol and e["uy"] <= tol and e["rho"] <= rho_tol and e[chi_key] <= chi_tol, (l, e)
    U.assert_walls_match(g, o, case["n_levels"] - 1, tol, rho_tol, U.reference_speed(case))
    # relative L2 differences per level (the form in which a converged-field
    # tolerance is often stated): the velocity vector within the velocity bound;
    # chi within its element-wise bound (FP32 measured 1.1e-5 to 3.0e-5: the
    # converged chi carries the FP32 rounding of the SA sources, see above)
    for l in range(case["n_levels"]):
        du = dn = dc = nc = 0.0
        for fg, fo in ((1, oracle.F_UX), (2, oracle.F_UY)):
            a, b = g.field(l, fg), o.field(l, fo)
            m = np.isfinite(b)
            du += float(np.sum((a[m] - b[m]) ** 2))
            dn += float(np.sum(b[m] ** 2))
        a, b = g.field(l, 3), o.field(l, oracle.F_CHI)
        m = np.isfinite(b)
        dc, nc = float(np.sum((a[m] - b[m]) ** 2)), float(np.sum(b[m] ** 2))
        ru, rc = np.sqrt(du / dn), np.sqrt(dc / nc)
        print(storage, "level", l, f"relative L2: u {ru:.2e} chi {rc:.2e}")
        assert ru <= tol and rc <= chi_tol, (l, ru, rc)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "mixed", "f16s", "bf16s", "mixeds"])
def test_converged_surface_data_per_storage(converged_oracle, storage):
    case, cpo, cfo, fo, _ = converged_oracle
    g = U.gpu_solver(case, storage)
    g.use_graph(True)
    g.advance(STEPS)
    cp, cf = g.surface(0)
    f = g.forces()
    e_cp = np.max(np.abs(cp - cpo))
    e_cf = np.max(np.abs(cf - cfo)) / np.max(np.abs(cfo))
    e_f = [abs(f[k] - fo[k]) / abs(fo[k]) for k in (2, 3)]
    print(f"{storage}: Cp {e_cp:.3e} Cf {e_cf:.3e} C_D {e_f[0]:.3e} C_L {e_f[1]:.3e}")
    assert np.all(np.isfinite(cp)) and np.all(np.isfinite(cf)) and np.all(np.isfinite(f))
    if storage in BOUNDS:
        bcp, bcf, bforce = BOUNDS[storage]
        assert e_cp <= bcp and e_cf <= bcf and max(e_f) <= bforce, (e_cp, e_cf, e_f)
    elif storage in MEETS_CF_BOUND:
        assert e_cf <= CF_BOUND, e_cf


THREE_STEPS = 3000


@pytest.fixture(scope="module")
def three_element_oracle():
    """The small three-element case (slat, main element and flap; 3 levels to
    c/64): 3,000 coarse steps, 2,000 past the end of the start-up ramp, where C_L
    has settled to within 5e-4 of its late values (a residual oscillation of that
    size remains)."""
    case = LI.case_three_element(finest_cells_per_chord=64, n_levels=3, domain_chords=8.0, band_finest=0.3,
                                 n_side=256)
    o = oracle.Sim(case)
    o.advance(THREE_STEPS)
    return case, [o.surface(b) for b in range(3)], o.forces()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "f16s", "mixeds", "bf16s"])
def test_three_element_surface_data_per_storage(three_element_oracle, storage):
    """Every body's surface data against the FP64 oracle with the bounds of the
    single airfoil: FP64 to rounding, FP32 within the FP32 bounds (measured Cp
    4e-6, Cf 1.5e-6 of max |Cf|, C_D 3e-6, C_L 1e-6), the shifted FP16 and mixed
    storages within the Cf bound of the equal-Cf comparison on each body
    (measured 0.2 % and 0.05 %); the other 16-bit formats are reported only."""
    case, ref, fo = three_element_oracle
    g = U.gpu_solver(case, storage)
    g.use_graph(True)
    g.advance(THREE_STEPS)
    f = g.forces()
    assert np.all(np.isfinite(f))
    e_f = [abs(f[k] - fo[k]) / abs(fo[k]) for k in (2, 3)]
    worst_cp = worst_cf = 0.0
    for b, (cpo, cfo) in enumerate(ref):
        cp, cf = g.surface(b)
        assert np.all(np.isfinite(cp)) and np.all(np.isfinite(cf))
        worst_cp = max(worst_cp, float(np.max(np.abs(cp - cpo))))
        worst_cf = max(worst_cf, float(np.max(np.abs(cf - cfo)) / np.max(np.abs(cfo))))
    print(f"three-element {storage}: Cp {worst_cp:.3e} Cf {worst_cf:.3e} C_D {e_f[0]:.3e} C_L {e_f[1]:.3e}")
    if storage in BOUNDS:
        bcp, bcf, bforce = BOUNDS[storage]
        assert worst_cp <= bcp and worst_cf <= bcf and max(e_f) <= bforce, (worst_cp, worst_cf, e_f)
    elif storage in MEETS_CF_BOUND:
        assert worst_cf <= CF_BOUND, worst_cf
