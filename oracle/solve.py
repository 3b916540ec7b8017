"""End-to-end oracle solve: build, precondition, FGMRES (test infrastructure)."""
import numpy as np

from . import comparators
from . import discretisation as dsc
from . import krylov, network


class Problem:
    """Oracle view of one problem: discretisation, RHS and (optionally) the network."""

    def __init__(self, prob, blob=None):
        self.D = dsc.Discretisation(prob)
        self.b = dsc.rhs(self.D)
        self.diag = dsc.diagonal(self.D)
        self.net = network.Net(blob) if blob is not None else None
        self.fields = network.coeffnet(self.net, self.D) if self.net is not None else None

    def apply(self, x):
        return dsc.apply_L(self.D, x).reshape(-1)

    def precond(self, v):
        return network.vcycle(self.net, self.fields, self.diag, v, self.D).reshape(-1)

    def precond_bf16(self, v):
        """The V-cycle with its convolution inputs and weights rounded to bfloat16."""
        return network.vcycle(self.net, self.fields, self.diag, v, self.D, bf16=True).reshape(-1)

    def block_jacobi(self, v):
        return comparators.block_jacobi(self.D, v).reshape(-1)

    def solve(self, rtol=1e-10, restart=30, max_iters=20000, use_net=True, record=None, precond=None):
        """precond: "net" (the default when a network is loaded), "bj" or "none"."""
        kind = precond if precond is not None else ("net" if (use_net and self.net is not None) else "none")
        M = {"net": self.precond, "bj": self.block_jacobi, "none": None}[kind]
        x, st = krylov.fgmres(self.apply, self.b.reshape(-1), M, restart, rtol, max_iters,
                              record=record)
        return x.reshape(self.D.N, self.D.cells), st


def relative_residual(P, x):
    r = P.b.reshape(-1) - P.apply(np.asarray(x).reshape(-1))
    return float(np.linalg.norm(r) / np.linalg.norm(P.b))
