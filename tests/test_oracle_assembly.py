"""Pins for the oracle's Nedelec assembly (eq. (5), eq. (8), Sec. 2.1)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.assemble import Discretisation


@pytest.fixture(scope="module")
def d4():
    return Discretisation(4, 2.0)


def test_curl_grad_is_zero(d4):
    """curl o grad = 0: the discrete gradients of interior hat functions lie
    in the kernel of K."""
    G = d4.discrete_gradient()
    KG = (d4.K @ G).toarray()
    assert np.abs(KG).max() <= 1e-13 * abs(d4.K).max()
    assert G.shape == (316, 27)


def test_symmetry_and_spd(d4):
    for M in (d4.K, d4.M, d4.A):
        assert abs(M - M.T).max() <= 1e-14 * abs(M).max()
    np.linalg.cholesky(d4.M.toarray())                  # M is SPD


def test_rank_of_curl_curl(d4):
    """rank K = #interior edges - #interior vertices (exact discrete sequence
    on the cube)."""
    assert np.linalg.matrix_rank(d4.K.toarray()) == 316 - 27


def test_inertia(d4):
    """kappa^2 = 4 lies below the first positive discrete curl-curl
    eigenvalue, so A = K - 4 M is negative exactly on the gradients:
    (n - 1)^3 = 27 negative eigenvalues."""
    ev = np.linalg.eigvalsh(d4.A.toarray())
    assert int(np.sum(ev < 0)) == 27
    assert np.min(np.abs(ev)) > 1e-8


def _closed_form_mass(a, b):
    """int over the unit cube of |a + b x x|^2."""
    S = np.full((3, 3), 0.25) + np.eye(3) * (1.0 / 3.0 - 0.25)
    xbar = np.full(3, 0.5)
    return a @ a + 2 * a @ np.cross(b, xbar) + b @ b - b @ S @ b


@pytest.mark.parametrize("n", [1, 2, 3])
def test_linear_fields_exact(n):
    """For E = a + b x x (in N_0 on every element) with edge values
    u_e = E(mid_e) . (p_head - p_tail): u^T K u = |curl E|^2 = 4 |b|^2 and
    u^T M u = int |E|^2, both exactly."""
    d = Discretisation(n, 1.0)
    rng = np.random.default_rng(n)
    m = d.mesh
    p = m.coords.astype(np.float64) / n
    tail, head = p[m.edges[:, 0]], p[m.edges[:, 1]]
    mid = 0.5 * (tail + head)
    for _ in range(3):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        E = a + np.cross(b, mid)
        u = np.einsum("ij,ij->i", E, head - tail)
        assert abs(u @ (d.K_full @ u) - 4 * b @ b) <= 1e-12 * (1 + b @ b)
        ref = _closed_form_mass(a, b)
        assert abs(u @ (d.M_full @ u) - ref) <= 1e-12 * ref


def test_cavity_eigenvalue_convergence():
    """The smallest positive Maxwell eigenvalue of the unit cube with perfect
    conductor walls is 2 pi^2 (triple); the discrete one converges at O(h^2)."""
    errs = []
    for n in (4, 8):
        d = Discretisation(n, 0.0)
        vals = sla.eigh(d.K.toarray(), d.M.toarray(), eigvals_only=True,
                        subset_by_value=(1.0, 40.0))
        pos = np.sort(vals)[:3]
        errs.append(np.max(np.abs(pos - 2 * np.pi ** 2)) / (2 * np.pi ** 2))
    assert errs[1] < 0.05
    assert errs[0] / errs[1] > 3.0


@pytest.mark.parametrize("n", [2, 4])
def test_load_of_constant_field(n):
    """<J, Phi_j> for a constant J, two ways.  Whitney forms reproduce a
    constant field exactly, J = sum over all edges of (J . (p_head - p_tail))
    Phi_e, so the load equals (M_full d)[interior] with d_e = J . (p_head -
    p_tail), the mass matrix pinned above.  And since div J = 0, the load
    is orthogonal to the gradients of interior hat functions: G^T b = 0."""
    d = Discretisation(n, 1.0)
    m = d.mesh
    p = m.coords.astype(np.float64) / n
    for J in (np.array([0.0, 0.0, 1.0]), np.array([0.3, -1.2, 0.7])):
        b = d.load(J)
        de = (p[m.edges[:, 1]] - p[m.edges[:, 0]]) @ J
        ref = (d.M_full @ de)[m.interior]
        assert np.abs(b - ref).max() <= 1e-14 * np.abs(ref).max()
        G = d.discrete_gradient()
        assert np.abs(G.T @ b).max() <= 1e-14 * np.abs(b).max()
        assert np.abs(b).max() > 0


@pytest.mark.parametrize("n,box,beta", [(2, (0, 0, 0, 1, 2, 1), 10.0), (3, (1, 0, 1, 3, 2, 3), 0.25),
                                        (4, (1, 1, 1, 3, 3, 3), 100.0)])
def test_coefficient_box_energy(n, box, beta):
    """Piecewise constant curl-curl coefficient (Sec. 2.1): for E = a + b x x
    the curl is the constant 2b, so u^T K_beta u = 4 |b|^2 sum_T beta_T |T|
    = 4 |b|^2 (1 + (beta - 1) |box|) with |box| the box's volume; the mass
    matrix does not change and K_beta still annihilates the gradients."""
    d = Discretisation(n, 1.0, box, beta)
    d1 = Discretisation(n, 1.0)
    vol_box = np.prod(np.subtract(box[3:], box[:3])) / n ** 3
    m = d.mesh
    p = m.coords.astype(np.float64) / n
    tail, head = p[m.edges[:, 0]], p[m.edges[:, 1]]
    mid = 0.5 * (tail + head)
    rng = np.random.default_rng(7 + n)
    for _ in range(3):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        u = np.einsum("ij,ij->i", a + np.cross(b, mid), head - tail)
        ref = 4 * (b @ b) * (1 + (beta - 1) * vol_box)
        assert abs(u @ (d.K_full @ u) - ref) <= 1e-12 * ref
    assert abs(d.M - d1.M).max() == 0
    G = d.discrete_gradient()
    if G.shape[1]:
        assert abs(d.K @ G).max() <= 1e-13 * abs(d.K).max()


def test_coefficient_box_special_cases():
    """beta = 1 on any box, or no box, is the plain matrix; beta on the whole
    cube scales K exactly."""
    d1 = Discretisation(3, 2.0)
    assert abs(Discretisation(3, 2.0, (0, 1, 0, 2, 3, 1), 1.0).A - d1.A).max() == 0
    dw = Discretisation(3, 2.0, (0, 0, 0, 3, 3, 3), 4.0)
    assert abs(dw.K - 4.0 * d1.K).max() <= 1e-15 * abs(d1.K).max() * 4
    assert np.array_equal(dw.A.indptr, d1.A.indptr) and np.array_equal(dw.A.indices, d1.A.indices)


def _gauss_mass_over_cubes(n, mask, a, b):
    """int over the flagged cubes of |a + b x x|^2 by 2-point Gauss per axis
    (exact for this quadratic)."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    h = 1.0 / n
    total = 0.0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if not mask[i + n * (j + n * k)]:
                    continue
                for gx in g:
                    for gy in g:
                        for gz in g:
                            x = np.array([(i + gx) * h, (j + gy) * h, (k + gz) * h])
                            e = a + np.cross(b, x)
                            total += (e @ e) * h ** 3 / 8.0
    return total


@pytest.mark.parametrize("mm", [1, 2])
def test_two_box_domain_fields(mm):
    """On the two-box domain: K G = 0, rank K = N - interior vertices (the
    exact sequence on a contractible domain with a connected boundary), and
    linear fields E = a + b x x integrated exactly: u^T K u = 4 |b|^2 |Omega|
    and u^T M u = int_Omega |E|^2 (tensor Gauss quadrature over the cubes)."""
    from paper_2211_11303_amd.inputs import two_box_mask
    n, mask = two_box_mask(mm)
    d = Discretisation(n, 1.0, mask=mask)
    G = d.discrete_gradient()
    assert abs(d.K @ G).max() <= 1e-13 * abs(d.K).max()
    if mm == 1:
        assert np.linalg.matrix_rank(d.K.toarray()) == d.N - G.shape[1]
    vol = mask.sum() / n ** 3
    assert abs(d.volumes.sum() - vol) <= 1e-14
    m = d.mesh
    p = m.coords.astype(np.float64) / n
    tail, head = p[m.edges[:, 0]], p[m.edges[:, 1]]
    mid = 0.5 * (tail + head)
    rng = np.random.default_rng(17 + mm)
    for _ in range(2):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        u = np.einsum("ij,ij->i", a + np.cross(b, mid), head - tail)
        ref = 4 * (b @ b) * vol
        assert abs(u @ (d.K_full @ u) - ref) <= 1e-12 * ref
        refm = _gauss_mass_over_cubes(n, mask, a, b)
        assert abs(u @ (d.M_full @ u) - refm) <= 1e-12 * refm
