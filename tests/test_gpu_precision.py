"""Jacobian entries kept in BF16 / FP16 (products, sums and PCG in FP32, block
inverses and PCG dots in FP64): the node transforms and the energies after a
whole frame are compared with the FP64 oracle, beside the all-FP32 run.

Bounds: one BF16 rounding is a relative error of at most 2^-9 per entry,
one FP16 rounding 2^-12; the Gauss-Newton step built from them differs from
the FP32 step by about that fraction of its size, and later iterations
correct most of it, so the final transforms are held to 1e-3 rad / 1e-4 m
(BF16) and 2e-4 rad / 2e-5 m (FP16), energies to 1e-2 / 1e-3 relative."""
import numpy as np
import pytest

from gpu_common import gpu_lib, se3_errors, stream_for
from oracle import solve as S

pytestmark = pytest.mark.gpu

BOUNDS = {0: (1e-4, 1e-5, 1e-4), 1: (1e-3, 1e-4, 1e-2), 2: (2e-4, 2e-5, 1e-3)}


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_jacobian_precision_against_the_oracle(swgn, scene_cache, name):
    s = scene_cache(name)
    want, tr = S.oracle_solve(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params, linear="pcg")
    e_ref = np.array(tr["e_data"]) + s.params.lambda_reg * np.array(tr["e_reg"])
    for dt, (ta, tp, te) in BOUNDS.items():
        st = stream_for(swgn, s, jac_dtype=dt)
        stats = st.solve_frame(s.depth)
        got = st.node_se3()
        st.close()
        ang, dpos = se3_errors(got, want, s.node_pos)
        e_gpu = np.array(stats["e_data"]) + s.params.lambda_reg * np.array(stats["e_reg"])
        rel = np.max(np.abs(e_gpu - e_ref) / np.abs(e_ref))
        print(f"{name} jac_dtype={dt}: rot {ang.max():.3e} rad, pos {dpos.max():.3e} m, energy {rel:.3e}")
        assert ang.max() < ta and dpos.max() < tp and rel < te, (dt, ang.max(), dpos.max(), rel)
