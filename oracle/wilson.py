"""The Wilson(-twisted-mass) Dirac operator, its even/odd blocks and the Schur
complement, in complex128 on whole-lattice arrays.

Fields are ``psi[t][z][y][x][colour][spin]`` (one right-hand side); links are
``U[t][z][y][x][mu][a][b]`` with mu = 0..3 = x, y, z, t.  The lattice is
periodic in all four directions (isPeriodic(L) = true, Fig. "id").

Operator (Fig. "dirac"), read in its gauge-covariant form (the backward link is
the adjoint of the forward link one site back, Fig. "id"):

    (D psi)(x) = psi(x) + 2 i kappa mu gamma_5 psi(x)
                 - kappa sum_d [ (1 - gamma_d) U_d(x) psi(x + d)
                               + (1 + gamma_d) U_d(x - d)^dagger psi(x - d) ]

so D = A - kappa H with A = 1 + 2 i kappa mu gamma_5 site-diagonal and H the
hopping matrix.  A colour matrix acts on the colour index and a spin matrix on
the spin index of each site's 3 x 4 block, i.e. (M_c (x) M_s) V = M_c V M_s^T
(Sec. 4.2).

Even/odd: parity(x) = (x + y + z + t) mod 2, even = 0 (the projections P_e,
P_o of Fig. "dirac").  Parity-restricted fields are whole-lattice arrays that
are zero on the other parity.
"""
import numpy as np

from .gamma import GAMMA5, P_MINUS, P_PLUS

# site axis of each direction in a [t][z][y][x] array
AXIS = (3, 2, 1, 0)


def site_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def dims_of(field):
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def parity_field(dims):
    """parity(x) as an integer array over the sites."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x + y + z + t) % 2


def project(psi, parity):
    """P_parity psi: keep the sites of one parity, zero the rest."""
    m = (parity_field(dims_of(psi)) == parity)
    return psi * m[..., None, None]


def spin_mul(mat, f):
    """Apply a 4x4 spin matrix to the spin index of every site: f M^T."""
    return f @ mat.T


def colour_mul(u, f):
    """Apply per-site 3x3 colour matrices to the colour index: U f."""
    return u @ f


def dagger3(u):
    return np.conj(np.swapaxes(u, -1, -2))


def shift_fwd(f, mu):
    """(S f)(x) = f(x + mu_hat), periodic."""
    return np.roll(f, -1, axis=AXIS[mu])


def shift_bwd(f, mu):
    """(S f)(x) = f(x - mu_hat), periodic."""
    return np.roll(f, 1, axis=AXIS[mu])


def hop(U, psi, dagger=False):
    """Hopping term H psi (dagger=False) or H^dagger psi (dagger=True).

    H psi(x)        = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
    H^dagger psi(x) = sum_mu (1 + g_mu) U_mu(x) psi(x+mu) + (1 - g_mu) U_mu(x-mu)^+ psi(x-mu)
    """
    out = np.zeros_like(psi)
    for mu in range(4):
        pf, pb = (P_PLUS[mu], P_MINUS[mu]) if dagger else (P_MINUS[mu], P_PLUS[mu])
        u = U[..., mu, :, :]
        out += spin_mul(pf, colour_mul(u, shift_fwd(psi, mu)))
        out += spin_mul(pb, colour_mul(dagger3(shift_bwd(u, mu)), shift_bwd(psi, mu)))
    return out


def apply_A(kappa, mu, psi, dagger=False):
    """Site-diagonal part A = 1 + 2 i kappa mu gamma_5 (A^dagger with dagger=True)."""
    c = 2j * kappa * mu * (-1 if dagger else 1)
    return psi + c * spin_mul(GAMMA5, psi)


def apply_Ainv(kappa, mu, psi, dagger=False):
    """A^{-1} = (1 - 2 i kappa mu gamma_5) / (1 + 4 kappa^2 mu^2), since gamma_5^2 = 1."""
    c = -2j * kappa * mu * (-1 if dagger else 1)
    return (psi + c * spin_mul(GAMMA5, psi)) / (1.0 + 4.0 * kappa * kappa * mu * mu)


def apply_D(U, kappa, mu, psi):
    return apply_A(kappa, mu, psi) - kappa * hop(U, psi)


def apply_Ddag(U, kappa, mu, psi):
    return apply_A(kappa, mu, psi, dagger=True) - kappa * hop(U, psi, dagger=True)


def hop_eo(U, psi, out_parity, dagger=False):
    """Block H_{p,1-p}: from the sites of parity 1-p of psi to the sites of parity p."""
    return project(hop(U, project(psi, 1 - out_parity), dagger), out_parity)


# --- Schur complement on the odd sites (template "schur", Sec. 2) -----------
# D in (even, odd) blocks: D11 = D22 = A, D12 = -kappa H_eo, D21 = -kappa H_oe.
# D11 is site-diagonal and inverted in closed form.

def schur(U, kappa, mu, psi_o, dagger=False):
    """S psi_o = (D22 - D21 D11^{-1} D12) psi_o = A psi_o - kappa^2 H_oe A^{-1} H_eo psi_o
    (S^dagger with dagger=True)."""
    t = hop_eo(U, psi_o, 0, dagger)
    t = apply_Ainv(kappa, mu, t, dagger)
    t = hop_eo(U, t, 1, dagger)
    return project(apply_A(kappa, mu, psi_o, dagger), 1) - kappa * kappa * t


def schur_source(U, kappa, mu, b):
    """b_hat = v2 - D21 D11^{-1} v1 = b_o + kappa H_oe A^{-1} b_e."""
    be = project(b, 0)
    return project(b, 1) + kappa * hop_eo(U, apply_Ainv(kappa, mu, be), 1)


def reconstruct_even(U, kappa, mu, b, x_o):
    """x1 = D11^{-1} (v1 - D12 x2) = A^{-1} (b_e + kappa H_eo x_o), with v1 = P_e b
    (the first assignment of v1; see the reading of the second one in the design notes)."""
    return apply_Ainv(kappa, mu, project(b, 0) + kappa * hop_eo(U, x_o, 0))


def hop_site(U, psi, site, dagger=False):
    """(H psi) at one site (x, y, z, t), computed directly from the definition:
    8 neighbour terms, each a spin projector times a colour link times the
    neighbour's 3x4 block.  Used to check sampled outputs of large lattices."""
    dims = dims_of(psi)
    x = list(site)
    out = np.zeros((3, 4), dtype=np.complex128)
    for mu in range(4):
        pf, pb = (P_PLUS[mu], P_MINUS[mu]) if dagger else (P_MINUS[mu], P_PLUS[mu])
        xf = list(x)
        xf[mu] = (x[mu] + 1) % dims[mu]
        xb = list(x)
        xb[mu] = (x[mu] - 1) % dims[mu]
        uf = U[x[3], x[2], x[1], x[0], mu]
        ub = U[xb[3], xb[2], xb[1], xb[0], mu]
        out += uf @ psi[xf[3], xf[2], xf[1], xf[0]] @ pf.T
        out += np.conj(ub.T) @ psi[xb[3], xb[2], xb[1], xb[0]] @ pb.T
    return out


def norm2(f):
    return float(np.vdot(f, f).real)


def inner(a, b):
    """(a | b) = sum conj(a) b."""
    return complex(np.vdot(a, b))


def plaquette(U):
    """Average real trace / 3 of the elementary plaquettes (a summary of how rough a
    gauge field is; 1 for unit links)."""
    tot, n = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            umu, unu = U[..., mu, :, :], U[..., nu, :, :]
            p = umu @ shift_fwd(unu, mu) @ dagger3(shift_fwd(umu, nu)) @ dagger3(unu)
            tot += np.trace(p, axis1=-2, axis2=-1).real.mean() / 3.0
            n += 1
    return tot / n
