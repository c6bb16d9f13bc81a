"""Storage precision against the FP64 oracle at a converged state (needs an MI355X).

The 3-level airfoil (finest c/64, Re 6e6, M 0.15, 10 degrees) is run for 4000
coarse steps, by which the oracle's force coefficients are steady to six
digits, with populations stored in FP64, FP32, FP16 and BF16 (shifted,
f_i - w_i; arithmetic in FP32 for the 16-bit formats, FP64 Newton and force
sums), and mixed (FP32 on the two finest levels, FP16 on level 0). Each
storage is checked against the oracle's surface Cp, Cf and forces:

  * FP64: rounding-order differences only (1e-9 relative; measured 6e-13,
    1e-13, 6e-14, 1.2e-13);
  * FP32: Cp max-abs 1e-4, Cf max-abs 1e-4 max|Cf|, C_D and C_L 1e-5 relative
    (measured 5.2e-6, 9.8e-7, 2.3e-7, 8.8e-7);
  * FP16: Cp 3e-2, Cf 1e-2 max|Cf| (the FP32 Cf bound of the study, which FP16
    meets here), C_D and C_L 6e-3 relative (measured 6.0e-3, 4.5e-3, 3.6e-3,
    1.4e-3);
  * BF16: Cp 0.2, Cf 5e-2 max|Cf|, C_D and C_L 8e-2 (measured 6.5e-2, 8.0e-3,
    2.3e-2, 2.1e-2);
  * mixed: Cp 1.2e-2, Cf 6e-3 max|Cf|, C_D and C_L 5.5e-3 (measured 4.4e-3,
    2.3e-3, 2.2e-3, 1.8e-3): FP16 on the coarsest level alone costs most of the
    FP16 error, so the pressure level set by the far field, not the wall layer,
    limits the 16-bit formats;
  * the same three 16-bit formats with the free-stream storage shift (the
    stored value is f_i - f_eq_i(rho_ref, U) instead of f_i - w_i):
    FP16 Cp 5.5e-3, Cf 1.4e-3, C_D and C_L 1.2e-3 (measured 2.2e-3, 5.5e-4,
    4.6e-4, 1.4e-4); BF16 Cp 4e-2, Cf 6e-3, C_D and C_L 1.2e-2 (measured
    1.5e-2, 2.3e-3, 4.9e-3, 3.4e-6); mixed Cp 3.5e-4, Cf 1e-4 (the FP32 Cf
    bound), C_D and C_L 2.5e-4 (measured 1.3e-4, 3.5e-5, 9.9e-5, 8.5e-5).

The 16-bit bounds are the measured errors with a margin of about 2.5: they
record how much accuracy each format gives up, so that a regression shows.
"""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle
from tests import parity_util as U

pytestmark = pytest.mark.gpu

STEPS = 4000
BOUNDS = {  # storage: (Cp max-abs, Cf max-abs / max|Cf|, C_D and C_L relative)
    "f64": (1e-9, 1e-9, 1e-9),
    "f32": (1e-4, 1e-4, 1e-5),
    "f16": (3e-2, 1e-2, 6e-3),
    "bf16": (0.2, 5e-2, 8e-2),
    "mixed": (1.2e-2, 6e-3, 5.5e-3),
    "f16s": (5.5e-3, 1.4e-3, 1.2e-3),
    "bf16s": (4e-2, 6e-3, 1.2e-2),
    "mixeds": (3.5e-4, 1e-4, 2.5e-4),
}


@pytest.fixture(scope="module")
def converged_oracle():
    case = LI.case_airfoil_small()
    o = oracle.Sim(case)
    o.advance(STEPS)
    cp, cf = o.surface(0)
    return case, cp, cf, o.forces()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "mixed", "f16s", "bf16s", "mixeds"])
def test_converged_surface_data_per_storage(converged_oracle, storage):
    case, cpo, cfo, fo = converged_oracle
    g = U.gpu_solver(case, storage)
    g.use_graph(True)
    g.advance(STEPS)
    cp, cf = g.surface(0)
    f = g.forces()
    bcp, bcf, bforce = BOUNDS[storage]
    print(f"{storage}: Cp {np.max(np.abs(cp - cpo)):.3e} Cf {np.max(np.abs(cf - cfo)) / np.max(np.abs(cfo)):.3e} "
          f"C_D {abs(f[2] - fo[2]) / abs(fo[2]):.3e} C_L {abs(f[3] - fo[3]) / abs(fo[3]):.3e}")
    assert np.all(np.isfinite(cp)) and np.all(np.isfinite(cf))
    assert np.max(np.abs(cp - cpo)) <= bcp
    assert np.max(np.abs(cf - cfo)) <= bcf * np.max(np.abs(cfo))
    for k in (2, 3):                                   # C_D, C_L
        assert abs(f[k] - fo[k]) <= bforce * abs(fo[k]), (k, f[k], fo[k])
