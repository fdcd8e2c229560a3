"""The initialisation across IRF lengths, origins and bin counts (Methods,
initialisation: the log-matched filter over the pooled photons of the window
around each pixel).  The branch and bound adds each photon's bound terms to
pairs of sub-blocks whose count and guard entries follow the IRF's length
and origin, and stages the weights with a zero padding; these cases run one
IRF sample to nearly a thousand, origins at both ends of the IRF, bin
counts off every power of two, and the largest bin count of the LDS path
with the next one (the search from global memory).  Counts and depths must equal the oracle's
exactly, intensities and background to rounding."""
import numpy as np
import pytest

from gpu_util import device_to_oracle, to_dev_u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

# (IRF, bins, origin override or -1 for the IRF's peak)
CASES = {
    "L1": (lambda: synth.gaussian_irf(0.3, 0), 257, -1),
    "L5": (lambda: synth.gaussian_irf(1.0, 2), 300, -1),
    "L19_o0": (lambda: synth.gaussian_irf(1.5, 9), 511, 0),
    "L19_oLast": (lambda: synth.gaussian_irf(1.5, 9), 513, 18),
    "L137": (lambda: synth.exgauss_irf(3.0, 10.0, -18, 118), 1023, -1),
    "L137_oLast": (lambda: synth.exgauss_irf(3.0, 10.0, -18, 118), 1025, 136),
    "L426": (lambda: synth.exgauss_irf(5.0, 60.0, -25, 400), 2049, -1),
    "L941": (lambda: synth.exgauss_irf(8.0, 200.0, -40, 900), 2000, -1),
    # the last bin count whose sub-block bounds the LDS path keeps, and the next
    "L19_T8192": (lambda: synth.gaussian_irf(1.5, 9), 8192, -1),
    "L19_T8193": (lambda: synth.gaussian_irf(1.5, 9), 8193, -1),
}


def scene(name, rows=20, cols=24):
    mk, T, origin = CASES[name]
    irf = mk()
    rng = np.random.default_rng(1000 + sorted(CASES).index(name))
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    d = 0.1 * T + 0.7 * T * (j + 0.3 * i) / (cols + 0.3 * rows)     # a tilted plane inside the bins
    r = rng.uniform(6.0, 12.0, (rows, cols))
    Z = synth.render(rng, irf, T, d[None], r[None], 3.0 / T)
    return irf, T, origin, Z


@pytest.mark.parametrize("name", sorted(CASES))
def test_init_matches_oracle_across_irf_shapes(name):
    irf, T, origin, Z = scene(name)
    rows, cols = Z.shape[:2]
    p = dict(dz=0.1, p_xy=1.0, r_min=1.0, r_init=1, k_init=3)
    O = oracle.Oracle(oracle.Model(irf.probs, T, origin), oracle.Params(**p))
    ctx = rt3d.Context(irf.probs, T, origin=origin, **p)
    off, ent = oracle.compact(Z[None])
    so = O.init(off, ent, oracle.State(1, rows, cols, 4))
    print(f"[gpu-init-shapes] {name}: L {len(irf.probs)}, T {T}, origin {origin}, {len(ent)} entries", flush=True)
    d = ctx.step(rt3d.STEP_INIT, None, to_dev_u32(off), to_dev_u32(ent), shape=(1, rows, cols))
    assert ctx.query().device_error == 0
    sg = device_to_oracle(d, 4)
    assert so.cnt.sum() > 0
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    np.testing.assert_array_equal(sg.t, so.t)
    np.testing.assert_allclose(sg.r, so.r, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sg.b, so.b, rtol=2e-6, atol=1e-12)
