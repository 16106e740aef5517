"""Property tests of the oracle (Hypothesis): invariants that must hold for any
lattice shape, links, kappa, mu and fields, drawn at random over small periodic
lattices.  They pin the oracle's operator, Schur blocks, storage rounding and
network to what the mathematics fixes, independently of how the oracle
computes them:

* D^dagger is the adjoint of D, and gamma_5 D gamma_5 = D^dagger at mu = 0
  (gamma_5-hermiticity of the Wilson operator);
* gauge covariance: D[U^Omega] (Omega psi) = Omega (D[U] psi) for a random
  SU(3) gauge transform Omega;
* the hop couples only opposite parities, and its two parity blocks add up to
  it;
* the "schur" template: for any x, with b = D x, the Schur system
  S x_o = b_hat holds and x_e is recovered from b and x_o;
* the F16S storage error of a site is at most half an FP16 ulp of its scale,
  and reconstruct-12 rebuilds an SU(3) matrix from its first two rows;
* the network is linear, and network_adjoint is its adjoint.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import latgen
from oracle import ptc, storage, wilson as W
from oracle.gamma import GAMMA5

DIMS = st.sampled_from([(2, 2, 2, 2), (4, 2, 2, 2), (2, 4, 2, 2), (2, 2, 4, 2), (2, 2, 2, 4), (4, 2, 4, 2)])
SEEDS = st.integers(min_value=0, max_value=2**16)
KAPPA = st.floats(min_value=0.0, max_value=0.25)
MU = st.floats(min_value=0.0, max_value=0.5)
SETTINGS = settings(max_examples=40, deadline=None, derandomize=True)


def field(seed, dims, salt=0):
    g = np.random.default_rng([seed, salt])
    shape = W.site_shape(dims) + (3, 4)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def links(seed, dims):
    return latgen.small_config(dims, seed=seed % 97, kind="haar")["U"]


def rel(a, b):
    return np.sqrt(W.norm2(a - b) / max(W.norm2(b), 1e-300))


@SETTINGS
@given(dims=DIMS, seed=SEEDS, kappa=KAPPA, mu=MU)
def test_ddag_is_the_adjoint_of_d(dims, seed, kappa, mu):
    U = links(seed, dims)
    u, v = field(seed, dims, 1), field(seed, dims, 2)
    lhs = W.inner(u, W.apply_D(U, kappa, mu, v))
    rhs = W.inner(W.apply_Ddag(U, kappa, mu, u), v)
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


@SETTINGS
@given(dims=DIMS, seed=SEEDS, kappa=KAPPA)
def test_gamma5_hermiticity(dims, seed, kappa):
    U = links(seed, dims)
    v = field(seed, dims, 3)
    g5 = lambda f: W.spin_mul(GAMMA5, f)
    assert rel(g5(W.apply_D(U, kappa, 0.0, g5(v))), W.apply_Ddag(U, kappa, 0.0, v)) <= 1e-13


@SETTINGS
@given(dims=DIMS, seed=SEEDS, kappa=KAPPA, mu=MU)
def test_gauge_covariance(dims, seed, kappa, mu):
    U = links(seed, dims)
    om = latgen.random_su3_field(seed, dims)   # Omega(x), [t][z][y][x][3][3]
    # U'_mu(x) = Omega(x) U_mu(x) Omega(x + mu)^dagger
    Ut = np.empty_like(U)
    for m in range(4):
        om_fwd = np.roll(om, -1, axis=W.AXIS[m])
        Ut[..., m, :, :] = om @ U[..., m, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    v = field(seed, dims, 4)
    rot = lambda f: om @ f   # colour rotation of every site's 3 x 4 block
    assert rel(W.apply_D(Ut, kappa, mu, rot(v)), rot(W.apply_D(U, kappa, mu, v))) <= 1e-13


@SETTINGS
@given(dims=DIMS, seed=SEEDS)
def test_hop_couples_opposite_parities(dims, seed):
    U = links(seed, dims)
    v = field(seed, dims, 5)
    for p in (0, 1):
        # a field on one parity hops only onto the other
        assert W.norm2(W.project(W.hop(U, W.project(v, p)), p)) <= 1e-24 * W.norm2(v)
    blocks = W.hop_eo(U, v, 0) + W.hop_eo(U, v, 1)
    assert rel(blocks, W.hop(U, v)) <= 1e-14


@SETTINGS
@given(dims=DIMS, seed=SEEDS, kappa=KAPPA, mu=MU)
def test_schur_template_on_any_solution(dims, seed, kappa, mu):
    U = links(seed, dims)
    x = field(seed, dims, 6)
    b = W.apply_D(U, kappa, mu, x)
    x_o = W.project(x, 1)
    b_hat = W.schur_source(U, kappa, mu, b)
    assert rel(W.schur(U, kappa, mu, x_o), b_hat) <= 1e-12
    assert rel(W.reconstruct_even(U, kappa, mu, b, x_o), W.project(x, 0)) <= 1e-12


@SETTINGS
@given(dims=DIMS, seed=SEEDS, scale=st.floats(min_value=1e-6, max_value=1e6))
def test_f16s_error_within_half_an_ulp_of_the_scale(dims, seed, scale):
    psi = scale * field(seed, dims, 7)
    q, s = storage.f16s_quantize(psi)
    back = storage.f16s_dequantize(q, s)
    # per site: every real within half an FP16 ulp (2^-11 relative, at most
    # 2^-11 of a value below 1) times the site's scale, plus the FP32 rounding
    err = np.abs(np.concatenate([(back - psi).real[..., None], (back - psi).imag[..., None]], -1))
    site_scale = np.asarray(s, dtype=np.float64)
    while site_scale.ndim < err.ndim:
        site_scale = site_scale[..., None]
    assert np.all(err <= site_scale * (2.0 ** -11 + 2.0 ** -20) + 1e-30)


@SETTINGS
@given(seed=SEEDS)
def test_reconstruct12_rebuilds_su3(seed):
    g = np.random.default_rng([seed, 8])
    u = latgen.haar_su3(g, 16)
    rebuilt = storage.reconstruct12(u[:, :2, :])
    assert np.abs(rebuilt - u).max() <= 1e-13


@SETTINGS
@given(dims=DIMS, seed=SEEDS, a=st.complex_numbers(max_magnitude=10, allow_nan=False, allow_infinity=False))
def test_network_is_linear_with_its_adjoint(dims, seed, a):
    U = links(seed, dims)
    rng = np.random.default_rng([seed, 9])
    hidden = 2
    w1 = rng.standard_normal((ptc.NPATH, hidden, 1, 4, 4)) + 1j * rng.standard_normal((ptc.NPATH, hidden, 1, 4, 4))
    w2 = rng.standard_normal((ptc.NPATH, 1, hidden, 4, 4)) + 1j * rng.standard_normal((ptc.NPATH, 1, hidden, 4, 4))
    w = (w1, w2)
    u, v = field(seed, dims, 10), field(seed, dims, 11)
    lin = ptc.network(U, w, a * u + v)
    assert rel(lin, a * ptc.network(U, w, u) + ptc.network(U, w, v)) <= 1e-12
    lhs = W.inner(u, ptc.network(U, w, v))
    rhs = W.inner(ptc.network_adjoint(U, w, u), v)
    assert abs(lhs - rhs) <= 1e-11 * (1 + abs(lhs))
