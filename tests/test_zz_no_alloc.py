"""The allocation-free V-cycle (rte_precond_apply_noalloc) against rte_precond_apply.

Both run the same kernels in the same order on the same inputs, so the bar is
bit-for-bit equality.  Two calls in a row share the library's device array:
a C2-sized V-cycle first, then a smaller one (64^2 cells, 16 directions), so
the second call runs over what the first left in the array.  A V-cycle whose
activations exceed the array is refused with RTE_ENOMEM.
"""
import numpy as np
import pytest

import problems
from gpu_util import model_for, say, torch_cuda
from rte_inputs import configs

pytestmark = pytest.mark.gpu


def _case(prob, seed):
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    model, _ = model_for(prob)
    op = api.Operator(prob, model=model)
    rng = np.random.default_rng(seed)
    v = torch.from_numpy(rng.standard_normal(op.n)).cuda()
    return model, op, v


@pytest.mark.parametrize("mode", ["bf16", "fp32"])
def test_noalloc_vcycle_equals_workspace_vcycle(mode):
    torch = torch_cuda()
    big = _case(configs.c2(0), 11)
    small = _case(problems.make(n=64, ndir=16, g=0.3, eps=0.02, seed=5,
                                mg=dict(c0=16, levels=3, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3,
                                        seed=21)), 12)
    for name, (model, op, v) in (("128^2 x 32, 4 levels", big), ("64^2 x 16, 3 levels", small)):
        say("noalloc", mode, name)
        z_ws = op.precond(model, v, mode=mode)
        z_na = op.precond_noalloc(model, v, mode=mode)
        torch.cuda.synchronize()
        a, b = z_ws.cpu().numpy(), z_na.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    # the first shape again, after the smaller call left its values in the array
    model, op, v = big
    z_ws = op.precond(model, v, mode=mode)
    z_na = op.precond_noalloc(model, v, mode=mode)
    torch.cuda.synchronize()
    assert np.array_equal(z_ws.cpu().numpy(), z_na.cpu().numpy())


def test_noalloc_refuses_a_vcycle_larger_than_its_array():
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    from paper_2604_23265_amd._lib import RTE_ENOMEM, RteError
    prob = problems.make(n=512, ndir=32, g=0.3, eps=0.02, seed=6,
                         mg=dict(c0=32, levels=2, nu_pre=1, nu_post=1, nu_coarse=1, coef_ch=3, seed=22))
    model, _ = model_for(prob)
    op = api.Operator(prob, model=model)
    assert op.precond_workspace(model) > 64 << 20
    v = torch.zeros(op.n, dtype=torch.float64, device="cuda")
    with pytest.raises(RteError) as ei:
        op.precond_noalloc(model, v, mode="bf16")
    assert ei.value.code == RTE_ENOMEM
    assert "scratch" in str(ei.value)
