"""The algebra the HIP kernels evaluate instead of the paper's formulas,
restated in FP64 and checked against the definitions (CPU only).

Section 3 defines, for a stencil (a, b, c) on nodes -1, 1, 3, the candidate
P = (3a + 6b - c)/8 and the indicator S = (b - a)^2 + (13/12)(a - 2b + c)^2
(eqs. p and 2Dsmoothness), the combined indicator D = S + w (four
neighbours) (eqs. 2DsmoothnessFinal and tezine) and the blend with
alpha = 1/(eps + D)^beta (eqs. alpha, IzrazOmega2d).  The kernels carry
scaled copies of samples and indicators so that fewer instructions reach the
same weights; these tests pin each rewrite to the definitions, so a slip in
a constant or a sign of the derivation fails here without a GPU.  (The GPU
parity tests compare the kernels themselves with the oracle.)
"""
import numpy as np
import pytest


def P(a, b, c):
    return (3 * a + 6 * b - c) / 8


def S(a, b, c):
    return (b - a) ** 2 + 13.0 / 12.0 * (a - 2 * b + c) ** 2


@pytest.fixture
def triples():
    rng = np.random.default_rng(11)
    return rng.standard_normal((3, 1000)) * np.array([[1.0], [2.0], [0.5]])


def test_forward_half_and_kappa_copies(triples):
    # the doubling keeps h = v/2 and s = kappa v with kappa^2 = 13/48:
    # the candidate is (h_a + h_b) + kCandS (s_a - 2 s_b + s_c), the
    # indicator over 4 is (h_b - h_a)^2 + (s_a - 2 s_b + s_c)^2
    a, b, c = triples
    kappa = np.float64(np.float32(0.52041649986653320))   # the kernel's constants, as stored in FP32
    cand_s = np.float64(np.float32(-0.24019223070763074))
    assert kappa == pytest.approx(np.sqrt(13.0 / 48.0), rel=1e-7)
    assert cand_s == pytest.approx(-1.0 / (8.0 * np.sqrt(13.0 / 48.0)), rel=1e-7)
    k = np.sqrt(13.0 / 48.0)
    ha, hb = a / 2, b / 2
    dds = k * a - 2 * k * b + k * c
    np.testing.assert_allclose((ha + hb) + (-1.0 / (8 * k)) * dds, P(a, b, c), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose((hb - ha) ** 2 + dds ** 2, S(a, b, c) / 4, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("w", [1.0 / 8.0, 0.25, 0.0])
def test_eps_folded_into_every_indicator(w):
    # eps_q = eps / (4 (1 + 4 w)) added to each quarter indicator gives
    # (eps + D)/4 for the own indicator with weight 1 and four neighbours
    # with weight w; the adjoint's eps * (3/13) / (1 + 4 w) gives (3/13)(eps + D)
    rng = np.random.default_rng(5)
    own, nb = rng.random(200), rng.random((4, 200))
    eps = 1e-3
    D = own + w * nb.sum(axis=0)
    eq = eps / (4 * (1 + 4 * w))
    np.testing.assert_allclose((own / 4 + eq) + w * (nb / 4 + eq).sum(axis=0), (eps + D) / 4, rtol=1e-14)
    eh = eps * (3.0 / 13.0) / (1 + 4 * w)
    np.testing.assert_allclose((3 * own / 13 + eh) + w * (3 * nb / 13 + eh).sum(axis=0), 3 * (eps + D) / 13,
                               rtol=1e-14)


def test_adjoint_scaled_indicator_and_its_derivatives(triples):
    # SI* = (3/13) S = gh f + ddh^2, gh = (b - a)/2, f = (12/13) gh,
    # ddh = (a - 2b + c)/2, with gradient (ddh - f, f - 2 ddh, ddh)
    a, b, c = triples
    gh, ddh = (b - a) / 2, (a - 2 * b + c) / 2
    f = 12.0 / 13.0 * gh
    np.testing.assert_allclose(gh * f + ddh ** 2, 3.0 / 13.0 * S(a, b, c), rtol=1e-13)
    grad = np.stack([ddh - f, f - 2 * ddh, ddh])
    h = 1e-6
    for i in range(3):
        up, dn = [t.copy() for t in triples], [t.copy() for t in triples]
        up[i] += h
        dn[i] -= h
        fd = 3.0 / 13.0 * (S(*up) - S(*dn)) / (2 * h)
        np.testing.assert_allclose(grad[i], fd, rtol=1e-6, atol=1e-7)


def test_line_adjoint_is_the_sum_of_its_two_stencils():
    # one line x[-1], x0, x1, x2 carries the forward stencil (x0, x1, x2) and
    # the backward one (x1, x0, x[-1]); the kernel's per-line form
    #   E = gs ddh, F = f (gs_f + gs_b),
    #   s0 = 3/8 gp_f + 3/4 gp_b + E_f - 2 E_b - F
    #   s1 = 3/4 gp_f + 3/8 gp_b - 2 E_f + E_b + F
    #   cf = -1/8 gp_f + E_f,  cb = -1/8 gp_b + E_b
    # equals the seeds times the gradients of P and (3/13) S of each stencil
    rng = np.random.default_rng(7)
    xm1, x0, x1, x2 = rng.standard_normal((4, 500))
    gpf, gsf, gpb, gsb = rng.standard_normal((4, 500))
    f = 12.0 / 13.0 * (x1 - x0) / 2
    ddf, ddb = (x0 - 2 * x1 + x2) / 2, (x1 - 2 * x0 + xm1) / 2
    ef, eb = gsf * ddf, gsb * ddb
    F = (gsf + gsb) * f
    s0 = 3 / 8 * gpf + 3 / 4 * gpb + ef - 2 * eb - F
    s1 = 3 / 4 * gpf + 3 / 8 * gpb - 2 * ef + eb + F
    cf, cb = -1 / 8 * gpf + ef, -1 / 8 * gpb + eb

    def stencil_grad(p, q, r, gp, gs):   # d/d(p, q, r) of gp P + gs (3/13) S
        ghs, dds = (q - p) / 2, (p - 2 * q + r) / 2
        fs = 12.0 / 13.0 * ghs
        return (3 / 8 * gp + gs * (dds - fs), 3 / 4 * gp + gs * (fs - 2 * dds), -1 / 8 * gp + gs * dds)

    fa, fb, fc = stencil_grad(x0, x1, x2, gpf, gsf)
    ba, bb, bc = stencil_grad(x1, x0, xm1, gpb, gsb)
    np.testing.assert_allclose(s0, fa + bb, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(s1, fb + ba, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cf, fc, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cb, bc, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("beta", [1.0, 2.0, 1.5])
def test_blend_seed_factors(beta):
    # du/dp_k = omega_k and du/dt_k = -beta omega_k (p_k - u)/t_k for
    # u = sum t_k^-beta p_k / sum t_k^-beta; p_k - u = sum_j omega_j (p_k - p_j)
    # and the omega_k (p_k - u) sum to zero (the kernel takes the fourth as
    # minus the sum of the other three)
    rng = np.random.default_rng(int(beta * 10))
    t = rng.random((4, 300)) * 2 + 0.01
    p = rng.standard_normal((4, 300))

    def blend(t, p):
        a = t ** -beta
        return (a * p).sum(axis=0) / a.sum(axis=0)

    u = blend(t, p)
    om = t ** -beta / (t ** -beta).sum(axis=0)
    e = np.stack([(om * (p[k] - p)).sum(axis=0) for k in range(4)])
    np.testing.assert_allclose(e, p - u, rtol=1e-12, atol=1e-12)
    oe = om * e
    np.testing.assert_allclose(oe[3], -(oe[0] + oe[1] + oe[2]), rtol=1e-9, atol=1e-13)
    h = 1e-6
    for k in range(4):
        tu, td = t.copy(), t.copy()
        tu[k] += h
        td[k] -= h
        np.testing.assert_allclose(-beta * oe[k] / t[k], (blend(tu, p) - blend(td, p)) / (2 * h), rtol=1e-5,
                                   atol=1e-8)
        pu, pd = p.copy(), p.copy()
        pu[k] += h
        pd[k] -= h
        np.testing.assert_allclose(om[k], (blend(t, pu) - blend(t, pd)) / (2 * h), rtol=1e-6, atol=1e-9)
