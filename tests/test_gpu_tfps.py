"""The TFPS operator (Sec. 2.2) on the GPU against the TFPS oracle, through the C ABI.

Layouts: the library keeps coefficients cell-major [cells][2N] and equations [cells][2][N];
the oracle keeps [2N][cells] and [2][N][cells]; the tests permute.  Both sides build the
same eigen-bases (ascending eigenvalues, max-norm 1, the same sign rule), so A itself is
compared: the right-hand side and A x element by element (FP64 within 1e-11 of the largest
value: the bases agree to about 1e-12; FP32 inputs or outputs within 1e-6), and, as a check
that does not depend on the basis, the oracle's solution alpha* of the sparse system gives a
GPU residual at rounding and GPU cell-centre values equal to the oracle's psi.
"""
import numpy as np
import pytest

import problems
from gpu_util import dev, host, say, torch_cuda
from oracle import tfps

pytestmark = pytest.mark.gpu


def _two_material(n=12, ndir=16):
    st = np.where((np.add.outer(np.arange(n) // 4, np.arange(n) // 4) % 2) == 0, 1.0, 20.0)
    return problems.make(n=n, ndir=ndir, g=0.6, eps=0.05, sigma_t=st, sigma_a=0.3, q=1.0, seed=8, inflow="left")


CASES = {
    "8x8_n8": lambda: problems.make(n=8, ndir=8, g=0.5, eps=0.5, seed=2, inflow="random"),
    "10x10_n12": lambda: problems.make(n=10, ndir=12, g=0.3, eps=0.2, seed=3, inflow="random"),
    "16x16_n16_eps1e-2": lambda: problems.make(n=16, ndir=16, g=0.5, eps=0.01, seed=4, inflow="left"),
    "16x16_n32": lambda: problems.make(n=16, ndir=32, g=0.7, eps=0.3, seed=5, inflow="random"),
    "two_material_12x12_n16": _two_material,
    "1x1_n8": lambda: problems.make(n=1, ndir=8, g=0.2, eps=0.7, seed=9, inflow="random"),
    "2x2_n8": lambda: problems.make(n=2, ndir=8, g=0.4, eps=0.3, seed=10, inflow="random"),
}
_cache = {}


def case(name):
    torch_cuda()
    if name not in _cache:
        from paper_2604_23265_amd import api
        prob = dict(CASES[name]())
        prob["scheme"] = "tfps"
        op = api.Operator(prob)
        T = tfps.TFPS(prob)
        _cache[name] = (op, T)
    return _cache[name]


def to_cell_major_unknowns(a, T):
    return np.asarray(a).reshape(2 * T.N, -1).T.reshape(-1)


def to_oracle_unknowns(a, T):
    return np.asarray(a).reshape(-1, 2 * T.N).T.reshape(-1)


def to_cell_major_eqs(y, T):
    return np.asarray(y).reshape(2 * T.N, -1).T.reshape(-1)


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name", list(CASES))
def test_tfps_rhs_and_apply_fp64(name):
    say("tfps case", name)
    op, T = case(name)
    assert op.info["scheme"] == 1 and op.n == 2 * T.N * T.I * T.I
    b = host(op.rhs())
    bref = to_cell_major_eqs(T.rhs(), T)
    assert rel_max(b, bref) <= 1e-12
    rng = np.random.default_rng(3)
    for _ in range(2):
        a = rng.standard_normal(T.n)
        y = host(op.apply(dev(to_cell_major_unknowns(a, T))))
        yref = to_cell_major_eqs(T.apply(a), T)
        say("  apply fp64 max-norm rel err %.3e" % rel_max(y, yref))
        assert rel_max(y, yref) <= 1e-11


@pytest.mark.parametrize("name", ["8x8_n8", "16x16_n32", "two_material_12x12_n16"])
def test_tfps_apply_fp32(name):
    say("tfps fp32 case", name)
    op, T = case(name)
    a = np.random.default_rng(5).standard_normal(T.n).astype(np.float32)
    yref = to_cell_major_eqs(T.apply(a.astype(np.float64)), T)
    y = host(op.apply(dev(to_cell_major_unknowns(a, T), "float32"))).astype(np.float64)
    say("  apply fp32 max-norm rel err %.3e" % rel_max(y, yref))
    assert rel_max(y, yref) <= 1e-6


@pytest.mark.parametrize("name", list(CASES))
def test_tfps_solution_residual_and_cell_values(name):
    """The oracle's alpha* (sparse LU) through the GPU residual and cell-centre evaluation:
    basis-independent quantities of the discretisation."""
    say("tfps solution case", name)
    op, T = case(name)
    al = T.solve()
    r = host(op.residual(dev(to_cell_major_unknowns(al, T))))
    bn = np.linalg.norm(T.rhs())
    say("  residual of the oracle solution %.3e" % (np.linalg.norm(r) / bn))
    assert np.linalg.norm(r) <= 1e-10 * bn
    psi = host(op.cell_values(dev(to_cell_major_unknowns(al, T))))
    psi_ref = T.psi_centres(al).reshape(-1)
    # element-wise against the sum of the magnitudes of the terms: in the diffusive regime
    # the coefficients are large and cancel, and each term carries the bases' ~1e-12 agreement
    a = np.abs(np.asarray(al).reshape(2 * T.N, -1))
    mag = (np.einsum("cmk,kc->mc", np.abs(T.L), T.e["centre"].T * a) + np.abs(T.chis)[None, :]).reshape(-1)
    worst = float(np.max(np.abs(psi - psi_ref) / mag))
    say("  cell values max-norm rel err %.3e, worst against the terms' magnitudes %.3e"
        % (rel_max(psi, psi_ref), worst))
    assert worst <= 1e-11


def test_tfps_apply_is_deterministic():
    torch = torch_cuda()
    op, T = case("16x16_n32")
    x = torch.randn(op.n, dtype=torch.float64, device="cuda")
    y1 = op.apply(x)
    y2 = op.apply(x)
    assert bool((y1 == y2).all())


def test_tfps_rejections():
    torch_cuda()
    from paper_2604_23265_amd import api
    from paper_2604_23265_amd._lib import RteError
    from gpu_util import model_for
    base = problems.make(n=8, ndir=8, g=0.5, eps=0.5, seed=2, inflow="random")
    # sigma_a = 0 leaves the particular solution undefined (Sec. 2.2 assumes sigma_a != 0)
    p = dict(problems.make(n=8, ndir=8, g=0.5, eps=0.5, sigma_a=0.0, seed=2), scheme="tfps")
    with pytest.raises(RteError):
        api.Operator(p)
    # three dimensions
    p3 = dict(problems.make(dim=3, n=4, ndir=8, g=0.5, eps=0.5, kind="sphere", seed=2), scheme="tfps")
    with pytest.raises(RteError):
        api.Operator(p3)
    # an MgNet model (it preconditions the upwind scheme)
    base16 = problems.make(n=8, ndir=16, g=0.5, eps=0.5, seed=2, inflow="random")
    model, _ = model_for(base16)
    with pytest.raises(RteError):
        api.Operator(dict(base16, scheme="tfps"), model=model)
    # preconditioned solves are refused
    op = api.Operator(dict(base, scheme="tfps"))
    with pytest.raises(RteError):
        op.solve(precond="bj")


@pytest.mark.parametrize("name", ["1x1_n8", "2x2_n8"])
def test_tfps_solve_through_the_krylov_path(name):
    """rte_solve runs on the TFPS operator (no preconditioner): on these tiny systems
    (n = 16 and 64) GMRES with a cycle as long as n spans the whole space, so the solve
    reaches rtol 1e-12 and its cell values match the oracle's sparse-LU psi."""
    say("tfps solve case", name)
    op, T = case(name)
    x, st = op.solve(precond="none", restart=min(64, T.n), rtol=1e-12, max_iters=2000)
    say("  stats", st)
    assert st["converged"] == 1
    psi = host(op.cell_values(x))
    psi_ref = T.psi_centres(T.solve()).reshape(-1)
    assert rel_max(psi, psi_ref) <= 1e-9
