"""Solvers on the GPU operator (Sec. 1.2) and Table 1 through it.

* extreme singular values by Lanczos on A^T A against the oracle's dense SVD;
* Table 1 (mu = 1 / sigma_min) for DB2 and sym2, 1D and 2D, through the fast
  operator (soft pin, as on the oracle side);
* generalised sampling (CGLS) against the oracle's dense least-squares
  solution, and the paper's Example 2: truncated Walsh series and GS with
  DB2 / DB4 / DB6 from the first 32 x 32 Walsh samples of
  f = cos(3 pi t1 / 2) sin(3 pi t2);
* PBDW: data consistency and the GS coefficients beyond the samples;
* QCBP by Chambolle-Pock: the same iteration on the oracle's dense matrix
  (iterates agree), feasibility and the l1 bound.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle import walsh
from oracle.filters import Symlet
from tests import inputs
from tests.conftest import read_golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _op(dim, nu, j, q, j0=None, dtype=torch.float64, omega=None):
    from oracle.filters import family
    from paper_2106_00554_amd.operator import Wh2Wav
    print(f"[solvers] dim={dim} nu={nu!r} j={j} q={q} j0={j0}", flush=True)
    return Wh2Wav(dim, j, q, int(nu), j0, dtype, omega, family=family(nu))


def _table1():
    rows = {}
    for ln in read_golden("table1_mu.txt"):
        name, dim, *vals = ln.split()
        rows[(name, int(dim))] = [float(v) for v in vals]
    return rows


@pytest.mark.parametrize("dim,nu,j,q", [(1, 2, 7, 1), (1, Symlet(4), 6, 2), (1, 8, 6, 1), (2, 2, 4, 1),
                                        (2, Symlet(5), 4, 1)])
def test_extreme_singular_values_match_dense_svd(dim, nu, j, q):
    from paper_2106_00554_amd import solvers
    cfg = op.Config(nu, j, q)
    A = op.matrix_1d(cfg) if dim == 1 else op.dense_2d(cfg)
    s = np.linalg.svd(A, compute_uv=False)
    smin, smax = solvers.extreme_singular_values(_op(dim, nu, j, q, cfg.j0))
    assert abs(smin - s.min()) < 1e-10 and abs(smax - s.max()) < 1e-10


def test_table1_db2_sym2_through_the_fast_operator():
    """Table 1's DB2 / sym2 rows: 1D M = 2^7 (q = 1..4) and 2D M = 32^2 (q = 1, 2)."""
    from paper_2106_00554_amd import solvers
    rows = _table1()
    for name, nu in (("DB2", 2), ("sym2", Symlet(2))):
        for q in (1, 2, 3, 4):
            smin, _ = solvers.extreme_singular_values(_op(1, nu, 7, q, 7))
            ref = rows[(name, 1)][q - 1]
            print(f"[table1] {name} 1D q={q}: mu {1 / smin:.4f} (paper {ref})", flush=True)
            assert abs(1 / smin - ref) / ref < 1.5e-3
        for q in (1, 2):
            smin, _ = solvers.extreme_singular_values(_op(2, nu, 5, q, 5))
            ref = rows[(name, 2)][q - 1]
            print(f"[table1] {name} 2D q={q}: mu {1 / smin:.4f} (paper {ref})", flush=True)
            assert abs(1 / smin - ref) / ref < 3e-3


def test_generalised_sampling_matches_dense_least_squares():
    from paper_2106_00554_amd import solvers
    cfg = op.Config(4, 4, 1, 3)
    A2 = op.dense_2d(cfg)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(A2.shape[0])
    ref, *_ = np.linalg.lstsq(A2, y, rcond=None)
    o = _op(2, 4, 4, 1, 3)
    z, hist = solvers.generalised_sampling(o, torch.tensor(y, device="cuda"), iters=300, tol=1e-13)
    got = z.cpu().numpy().reshape(-1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9, hist[-3:]


def _example2_samples(N):
    """<f, w_n1 (x) w_n2> for n1, n2 < N, f = cos(3 pi t1 / 2) sin(3 pi t2): exact cell integrals
    of the separable factors (closed form) against the Walsh matrix of Def. 3.1."""
    i = np.arange(N)
    c1 = (np.sin(1.5 * np.pi * (i + 1) / N) - np.sin(1.5 * np.pi * i / N)) / (1.5 * np.pi)
    c2 = (np.cos(3 * np.pi * i / N) - np.cos(3 * np.pi * (i + 1) / N)) / (3 * np.pi)
    H = walsh.walsh_matrix(int(np.log2(N)))
    return np.outer(H @ c1, H @ c2), c1, c2


def _relative_error_from_walsh(alpha, c1, c2, Nf):
    """||f - g|| / ||f|| on the cells of side 1 / Nf, g given by its Walsh coefficients alpha (Nf x Nf)
    and f by the cell integrals c1 (x) c2 at the same resolution (cell averages compared)."""
    J = int(np.log2(Nf))
    H = walsh.walsh_matrix(J)
    g_cells = H.T @ alpha @ H / Nf ** 2          # cell integrals of g (H H^T = Nf I)
    f_cells = np.outer(c1, c2)
    return np.linalg.norm(g_cells - f_cells) / np.linalg.norm(f_cells)


def test_example2_truncated_walsh_and_generalised_sampling():
    """Example 2 (Sec. 6): relative errors 0.0950 (truncated Walsh), then GS with DB2, DB4, DB6
    from the first 32 x 32 Walsh samples decreasing with nu.  The error is measured on 256^2 cells
    (the paper evaluates in many points); the GS space is M = 16^2 (q = 1, not stated)."""
    from paper_2106_00554_amd import solvers
    N, Nf = 32, 256
    y2, _, _ = _example2_samples(N)
    _, c1f, c2f = _example2_samples(Nf)
    # truncated Walsh series: its Walsh coefficients are y below 32 and 0 beyond
    alpha = np.zeros((Nf, Nf))
    alpha[:N, :N] = y2
    tw = _relative_error_from_walsh(alpha, c1f, c2f, Nf)
    print(f"[example2] truncated Walsh {tw:.4f} (paper 0.0950)", flush=True)
    assert abs(tw - 0.0950) < 1.5e-3
    errs = {}
    for nu in (2, 4, 6):
        j, q = 4, 1
        o = _op(2, nu, j, q, 4 if nu == 6 else None)
        z, hist = solvers.generalised_sampling(o, torch.tensor(y2.reshape(-1), device="cuda"), iters=400,
                                               tol=1e-12)
        # Walsh coefficients of the reconstruction up to Nf from an operator with more samples
        big = _op(2, nu, j, int(np.log2(Nf)) - j, o.j0)
        a_f = big.forward(z).cpu().numpy().reshape(Nf, Nf)
        errs[nu] = _relative_error_from_walsh(a_f, c1f, c2f, Nf)
        print(f"[example2] GS DB{nu}: {errs[nu]:.4f}", flush=True)
    print("[example2] paper: DB2 0.0518, DB4 0.0290, DB6 0.0215", flush=True)
    assert tw > errs[2] > errs[4] > errs[6]


def test_pbdw_is_data_consistent():
    from paper_2106_00554_amd import solvers
    N, K, j = 32, 128, 4
    y2, _, _ = _example2_samples(N)
    o = _op(2, 4, j, 1)
    z, _ = solvers.generalised_sampling(o, torch.tensor(y2.reshape(-1), device="cuda"), iters=400)
    big = _op(2, 4, j, 3)
    n1, n2 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    first = torch.tensor((n1 * K + n2).reshape(-1), device="cuda")
    w = solvers.pbdw(big, z, torch.tensor(y2.reshape(-1), device="cuda"), first).cpu().numpy().reshape(K, K)
    gs = big.forward(z).cpu().numpy().reshape(K, K)
    assert np.array_equal(w[:N, :N], y2)
    mask = np.ones((K, K), bool)
    mask[:N, :N] = False
    assert np.array_equal(w[mask], gs[mask])


def test_qcbp_chambolle_pock_matches_dense_iteration():
    from paper_2106_00554_amd import solvers
    cfg = op.Config(2, 4, 1, 2)
    A2 = op.dense_2d(cfg)
    x_true = inputs.coefficients_2d(4, 2, 11, zero_frac=0.9)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.3, 12, core=4)
    A = A2[omega]
    y = A @ x_true.reshape(-1)
    eta = (0.01 * np.linalg.norm(y)) ** 2
    # the same iteration on the dense matrix
    tau = sigma = 0.99
    z = np.zeros(A.shape[1])
    zbar, p = z.copy(), np.zeros(A.shape[0])
    for _ in range(300):
        v = p + sigma * (A @ zbar)
        u = v / sigma - y
        p = v - sigma * (y + min(1.0, np.sqrt(eta) / max(np.linalg.norm(u), 1e-300)) * u)
        t = z - tau * (A.T @ p)
        z_new = np.sign(t) * np.maximum(np.abs(t) - tau, 0)
        zbar, z = 2 * z_new - z, z_new
    o = _op(2, 2, 4, 1, 2, omega=omega)
    zg = solvers.qcbp(o, torch.tensor(y, device="cuda"), eta, iters=300).cpu().numpy().reshape(-1)
    assert np.linalg.norm(zg - z) / np.linalg.norm(z) < 1e-9
    # longer run: feasible and no larger in l1 than the (feasible) true coefficients
    zl = solvers.qcbp(o, torch.tensor(y, device="cuda"), eta, iters=3000).cpu().numpy().reshape(-1)
    assert np.linalg.norm(A @ zl - y) ** 2 <= eta * 1.05
    assert np.abs(zl).sum() <= np.abs(x_true).sum() * 1.01
