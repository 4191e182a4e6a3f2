"""Split-BF16 contraction (DG_BF16X3, N = 5..7) against the FP64 oracle, through the C ABI.

Bound, derived from the arithmetic. Each operand and operator value x is split into
x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest, u = 2^-9 for bf16's 8-bit
significand), and x y is taken as x_hi y_hi + x_hi y_lo + x_lo y_hi, so per product
    |x y - product| <= |x_lo y_lo| + |x - x_hi - x_lo| |y| + |x_hi| |y - y_hi - y_lo|
                    <= 3 u^2 (1 + u)^2 |x y|                  (about 1.1e-5 |x y|),
and the FP32 sum of KD such products adds at most KD 2^-24 of the sum of their magnitudes.
So at every node
    |rhs_gpu - rhs| <= beta * A,  beta = 2 (3 u^2 + KD 2^-24)  (a factor 2 of margin),
where A is the same contraction in absolute values: sum_mu |D_mu| (|c_mu,b| |V_c| +
|c_mu,c| |V_b|) + |LIFT| |Fscale flux| (V the fields feeding the curl, c the inverse-map
derivatives), divided by eps or mu in a medium; the FP32 state, fluxes and operand add
1e-6 max |rhs| at most. One RK step: |u_gpu - u| <= 5 dt beta max A + 1e-6 max |u|.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import gpu_rhs, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9


def kd(N):
    Np, Nf4 = (N + 1) * (N + 2) * (N + 3) // 6, 2 * (N + 1) * (N + 2)
    np8, nf8 = -(-Np // 8) * 8, -(-Nf4 // 8) * 8
    return -(-(3 * np8 + nf8) // 32) * 32


def beta(N):
    return 2.0 * (3 * U_BF16 ** 2 * (1 + U_BF16) ** 2 + kd(N) * 2.0 ** -24)


def abs_contraction(m, u, elems, **kw):
    """A: the right-hand side's contraction in absolute values at the elements `elems`."""
    ref = m.ref
    G = m.G[elems]                       # (k, mu, nu) = d r_mu / d x_nu
    ue = np.abs(u[:, elems])
    out = np.zeros((6, len(elems), ref.Np))
    D = (np.abs(ref.Dr), np.abs(ref.Ds), np.abs(ref.Dt))
    for f in range(6):
        a = f % 3
        b, c = (a + 1) % 3, (a + 2) % 3
        src = 3 if f < 3 else 0
        for mu in range(3):
            op = np.abs(G[:, mu, b])[:, None] * ue[src + c] + np.abs(G[:, mu, c])[:, None] * ue[src + b]
            out[f] += op @ D[mu].T
    fl = W.surface_flux(m, u, **{k: v for k, v in kw.items() if k in ("eps", "mu", "absorb", "scatter", "incident", "t")})
    F = np.abs(fl[:, elems] * m.Fscale[elems][None, :, :, None]).reshape(6, len(elems), -1)
    out += F @ np.abs(ref.LIFT).T
    if "eps" in kw:
        out[:3] /= np.asarray(kw["eps"])[elems][None, :, None]
        out[3:] /= np.asarray(kw["mu"])[elems][None, :, None]
    return out


def _bf16x3_case(N, n, medium, shuffle=True):
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=shuffle)
    m = Mm.Mesh(v, e, R.ref_element(N))
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32")
    kw, skw = {}, {}
    if medium:
        eps, mu = dginputs.random_materials(m.K, seed=31)
        f = dginputs.faces_on_plane
        fb = (2 * f(v, e, 2, 1.0)).astype(np.int8)
        kw = dict(eps=eps, mu=mu, absorb=f(v, m.etov, 2, 1.0).astype(bool))
        skw = dict(eps=eps, mu=mu, face_bc=fb)
    return v, e, m, u, kw, skw


@pytest.mark.parametrize("medium", [False, True])
@pytest.mark.parametrize("N", [5, 6, 7])
def test_bf16x3_within_derived_bound(N, medium):
    v, e, m, u, kw, skw = _bf16x3_case(N, 3, medium)
    say(f"case: bf16x3 N={N} K={m.K} {'medium' if medium else 'vacuum'}")
    s = P.Solver(v, e, N, "bf16x3", **skw)
    elems = np.arange(m.K)
    A = abs_contraction(m, u, elems, **kw)
    r, ro = gpu_rhs(s, u), W.rhs(m, u, **kw)
    lim = beta(N) * A + 1e-6 * np.max(np.abs(ro))
    worst = float(np.max(np.abs(r - ro) / lim))
    say(f"  rhs rel L2 {rel_l2(r, ro):.2e}; worst |err| / bound {worst:.3f} (beta {beta(N):.2e})")
    assert worst <= 1.0
    dt = W.stable_dt(m)
    s.set_fields(u)
    s.rk_step(dt)
    uo, _ = W.lsrk4_step(m, u, dt, **kw)
    ug = s.get_fields()
    lim1 = 5 * dt * beta(N) * np.max(A) + 1e-6 * np.max(np.abs(uo))
    say(f"  1 step rel L2 {rel_l2(ug, uo):.2e}; worst |err| / bound {np.max(np.abs(ug - uo)) / lim1:.3f}")
    assert np.max(np.abs(ug - uo)) <= lim1
    # the split matters: a plain FP32 contraction is closer to the oracle
    s32 = P.Solver(v, e, N, "f32", **skw)
    assert rel_l2(gpu_rhs(s32, u), ro) < rel_l2(r, ro)
    s.free()
    s32.free()


@pytest.mark.parametrize("N,n", [(5, 31), (7, 25)])
def test_bf16x3_full_size_steady_state_loop(N, n):
    """N = 5 on 6 * 31^3 = 178,746 and N = 7 on 6 * 25^3 = 93,750 shuffled tets (8-element
    tiles, a ragged last one, many tiles per persistent workgroup): sampled right-hand side
    within the bound."""
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=True)
    m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32")
    say(f"case: bf16x3 N={N} K={m.K} full size")
    s = P.Solver(v, e, N, "bf16x3")
    g = np.random.default_rng(77)
    sample = np.unique(np.concatenate([g.choice(m.K, 400, replace=False), [0, m.K - 1]]))
    r = gpu_rhs(s, u)[:, sample]
    ro = W.rhs_at(m, u, sample)
    # absolute contraction at the sampled elements, with their face fluxes from rhs_at's maps
    ref = m.ref
    Gm = m.G[sample]
    ue = np.abs(u[:, sample])
    A = np.zeros_like(ro)
    D = (np.abs(ref.Dr), np.abs(ref.Ds), np.abs(ref.Dt))
    for f in range(6):
        a = f % 3
        b, c = (a + 1) % 3, (a + 2) % 3
        src = 3 if f < 3 else 0
        for mu in range(3):
            A[f] += (np.abs(Gm[:, mu, b])[:, None] * ue[src + c] + np.abs(Gm[:, mu, c])[:, None] * ue[src + b]) @ D[mu].T
    # the lift part is bounded through the sampled fluxes recovered from the oracle's split:
    # rhs - volume = LIFT (Fscale flux); bound |LIFT| |Fscale flux| by the face values
    from oracle.mesh import face_maps
    vM, vP = face_maps(m.x, m.EToE, m.EToF, ref.Fmask, sample)
    flat = u.reshape(6, -1)
    jump = np.abs(flat[:, vP]) + np.abs(flat[:, vM])            # |u+| + |u-| >= |[u]|
    Fb = (jump.sum(0, keepdims=True) * m.Fscale[sample][None, :, :, None]).reshape(1, len(sample), -1)
    A += Fb @ np.abs(ref.LIFT).T                                 # each flux component <= sum |[u]| Fscale
    lim = beta(N) * A + 1e-6 * np.max(np.abs(ro))
    worst = float(np.max(np.abs(r - ro) / lim))
    say(f"  sampled rhs rel L2 {rel_l2(r, ro):.2e}; worst |err| / bound {worst:.3f}")
    assert worst <= 1.0
    s.free()
