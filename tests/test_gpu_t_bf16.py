"""BF16 storage of the V-cycle's t tensors (the modulated residuals and a^{-1} (.) f, which only
ever feed convolutions) gives bitwise the V-cycle of FP32 storage.

The convolutions round their inputs to bfloat16 when they stage them; storing t as bfloat16
moves that rounding to where t is produced, on the same FP32 value, so nothing else may
change.  Each case runs rte_precond_apply twice on the same input, with RTE_T_BF16=0 (every t
in FP32) and with the default (t in BF16 on the levels whose producers and consumers all run
on the tiled 2D kernel), and requires equal bits.  The cases cover: every level in BF16 (the
C2 instance with the trained weights); a first level of 16 channels that stays FP32 while the
coarser ones switch; no pre-smoothing (the restriction reads f in FP32 and writes t in BF16);
one pre-smoothing step (the restriction reads the residual t); no coarse smoothing (the
restriction writes no t); grids of one 8x8 patch at the coarsest level.  Each launch form's
FP32-storage twin is compared with the oracle in test_gpu_conv_parity.py.
"""
import os

import numpy as np
import pytest

import problems
from gpu_util import dev, host, model_for, say, torch_cuda
from rte_inputs import configs

pytestmark = pytest.mark.gpu


def _mg(c0, levels, pre, post, coarse, seed):
    return dict(c0=c0, levels=levels, nu_pre=pre, nu_post=post, nu_coarse=coarse, coef_ch=3, seed=seed)


CASES = {
    "c2_trained": None,
    "c2_small_c16": lambda: configs.c2(0, n=32, ndir=16, levels=3),
    "no_presmoothing": lambda: problems.make(n=32, ndir=16, g=0.5, eps=0.05, inflow="random", seed=41,
                                             mg=_mg(32, 3, 0, 2, 2, 141)),
    "one_presmoothing": lambda: problems.make(n=64, ndir=16, g=0.3, eps=0.02, inflow="left", seed=42,
                                              mg=_mg(32, 4, 1, 1, 1, 142)),
    "no_coarse_smoothing": lambda: problems.make(n=32, ndir=8, g=0.6, eps=0.1, inflow="random", seed=43,
                                                 mg=_mg(32, 3, 2, 2, 0, 143)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_bf16_t_storage_is_bitwise_fp32_storage(name):
    torch_cuda()
    from paper_2604_23265_amd import api
    say("case t storage", name)
    if name == "c2_trained":
        prob = configs.c2(0)
        path = os.path.join(os.path.dirname(api.__file__), "weights", "c2_mgnet.mgn1")
        model = api.Model(open(path, "rb").read())
    else:
        prob = CASES[name]()
        model, _ = model_for(prob)
    op = api.Operator(prob, model=model)
    v = np.random.default_rng(17).standard_normal(op.n)
    os.environ["RTE_T_BF16"] = "0"
    try:
        z32 = host(op.precond(model, dev(v), mode="bf16"))
    finally:
        os.environ.pop("RTE_T_BF16", None)
    z16 = host(op.precond(model, dev(v), mode="bf16"))
    say("  max |z| %.3e, elements differing %d" % (np.max(np.abs(z32)), int(np.sum(z32 != z16))))
    assert np.array_equal(z32, z16)
