"""dg_energy_noalloc (the allocation-free energy call) against dg_energy, through the C ABI.

Two calls in a row on two handles, the second with the smaller mesh, so that the static scratch
array holds the first call's partial sums when the second one runs; then the first handle again.
The two calls sum their partial energies in different orders (tree against sequential), so
they agree to rounding: relative 1e-13 in the FP64 accumulator.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import say
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu


def _solver(n, N, prec, medium):
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
    u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    kw = {}
    if medium:
        kw["eps"], kw["mu"] = dginputs.random_materials(m.K, seed=7)
    s = P.Solver(v, e, N, prec, **kw)
    s.set_fields(u.astype(s.dtype))
    return s


def test_energy_noalloc_matches_energy_on_two_calls():
    import torch
    big = _solver(11, 3, "f64", medium=True)     # 7,986 elements: 125 partial sums
    small = _solver(4, 4, "f32", medium=False)   # 384 elements: 6 partial sums
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for s, slot in ((big, 0), (small, 1)):
        say(f"case: energy_noalloc K={s.K} N={s.order} {s.precision}")
        s.energy_noalloc(out[slot:])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array([big.energy(), small.energy()])
    say(f"  noalloc {got}, energy {want}")
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - want) / want) <= 1e-13
    # the first handle again, after the smaller call left its partial sums in the scratch
    again = torch.zeros(1, dtype=torch.float64, device="cuda")
    big.energy_noalloc(again)
    torch.cuda.synchronize()
    assert abs(again.item() - want[0]) <= 1e-13 * want[0]
    big.free()
    small.free()


def test_energy_noalloc_argument_errors():
    import torch
    v, e = dginputs.kuhn_cube(1)
    host_only = P.Solver(v, e, 2, "f64", device=-1)
    rc = P.lib().dg_energy_noalloc(host_only._h, None, None)
    assert rc == -6   # DG_E_STATE: no device state
    s = P.Solver(v, e, 2, "f64")
    assert P.lib().dg_energy_noalloc(s._h, None, None) == -1   # DG_E_ARG: NULL output
    with pytest.raises(P.DGError):
        s.energy_noalloc(torch.zeros(1, dtype=torch.float32, device="cuda"))
    s.free()
