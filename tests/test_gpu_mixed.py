"""Mixed precision (FP32 Householder QR with FP64 reflector norms, FP64
refinement against the FP64 stacked matrix): c within 1e-8 of the FP64 oracle,
with the error reported per refinement step."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import GpuFit, log

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-8


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _case(orc, n_configs, atoms, d, M, zeta, seed):
    inp = synth.make_fit_inputs(n_configs=n_configs, atoms=atoms, d=d, M=M, seed=seed)
    y = oracle.targets(orc, inp, zeta)
    ref = orc.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, jitter=1e-8, keep=True)
    assert ref.status == 0
    return inp, y, ref


def _mixed(inp, y, zeta, iters, tol=1e-14):
    from paper_2207_03803_amd import gap

    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, precision=gap.GAP_MIXED_FP32,
               max_refine_iters=iters, refine_tol=tol)
    g.build()
    g.h.solve(g.y, g.c, info=False)  # a capped run may end in GAP_ENOCONV: read it with sync()
    s, info = g.h.sync()
    return g, (s, info)


@pytest.fixture(scope="module")
def orc_m():
    return oracle.Oracle()


@pytest.mark.parametrize("name,args", [
    ("tiny", (200, (8, 64), 64, 256, 2, 0)),
    ("ragged", (400, (16, 64), 96, 333, 4, 3)),
    ("mid-size d=400 zeta=4", (2000, (16, 64), 400, 520, 4, 5)),
])
def test_mixed_refines_to_fp64_accuracy(orc_m, name, args):
    from paper_2207_03803_amd import gap

    inp, y, ref = _case(orc_m, *args)
    zeta = args[4]
    errs = []
    for k in (1, 2, 3, 5):
        g, _ = _mixed(inp, y, zeta, k, tol=0.0)  # tol 0: run exactly k steps
        errs.append(rel(g.c.cpu().numpy(), ref.c))
    g, (s, info) = _mixed(inp, y, zeta, 20, tol=1e-14)
    assert s == gap.GAP_OK
    c = g.c.cpu().numpy()
    err = rel(c, ref.c)
    log(f"  {name}: c rel err after 1,2,3,5 steps {['%.1e' % e for e in errs]}; "
        f"converged in {info.refine_iters} steps to {err:.2e} (last |dc|/|c| {info.step_rel:.1e}, eta {info.grad_rel:.1e})")
    assert info.device_status == gap.GAP_OK
    assert info.grad_rel <= 1e-13  # normal equations of the FP64 A (zero loss gradient)
    assert info.est_err == -1.0    # not requested
    assert info.cgls_iters == 0  # well within FP32's reach: corrected semi-normal equations alone
    assert err <= TOL_MIXED
    assert abs(info.residual_norm2 - ref.loss_tail) <= 1e-8 * ref.loss_tail


@pytest.mark.parametrize("sigma_per_atom", [1e-4, 3e-5])
def test_ill_conditioned_fit_moves_to_cgls(orc_m, sigma_per_atom):
    """M > N_c and a small sigma_E: kappa(A) of 1e7..1e8, where FP32's R makes the
    corrected semi-normal equations contract slowly or diverge.  The refinement
    moves to R-preconditioned CGLS and still reaches the oracle's c within the
    FP64 perturbation bound of the least-squares problem,
    u (kappa + kappa^2 ||r|| / (||A|| ||c||)) up to a small constant."""
    from paper_2207_03803_amd import gap

    inp = synth.make_fit_inputs(n_configs=600, atoms=(8, 64), d=128, M=800, seed=7, sigma_per_atom=sigma_per_atom)
    y = oracle.targets(orc_m, inp, 2)
    ref = orc_m.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 2, jitter=1e-8, keep=True)
    assert ref.status == 0
    sv = np.linalg.svd(np.triu(ref.A[:800]), compute_uv=False)  # A's singular values are R's
    kappa = sv[0] / sv[-1]
    rn = np.sqrt(ref.loss_tail)
    cn = np.linalg.norm(ref.c)
    bound = 32 * (np.finfo(np.float64).eps / 2) * (kappa + kappa ** 2 * rn / (sv[0] * cn))
    g, (s, info) = _mixed(inp, y, 2, 60, tol=1e-12)
    c = g.c.cpu().numpy()
    err = rel(c, ref.c)
    log(f"  sigma_E/atom {sigma_per_atom:g}: kappa(A) {kappa:.2e}; {info.refine_iters} steps, "
        f"{info.cgls_iters} of them CGLS; c rel err {err:.2e} (bound {bound:.1e}); last |dc|/|c| {info.step_rel:.1e}, eta {info.grad_rel:.1e}")
    assert s == gap.GAP_OK
    assert kappa > 5e6
    assert info.cgls_iters > 0
    assert err <= max(bound, TOL_MIXED)
    assert abs(info.residual_norm2 - ref.loss_tail) <= 1e-8 * ref.loss_tail


def test_mixed_reports_no_convergence(orc_m):
    """An unattainable tolerance within one step: GAP_ENOCONV, c still improved."""
    from paper_2207_03803_amd import gap

    inp, y, ref = _case(orc_m, 200, (8, 64), 64, 256, 2, 0)
    g, (s, info) = _mixed(inp, y, 2, 1, tol=0.0)
    assert s == gap.GAP_ENOCONV
    assert info.refine_iters == 1
