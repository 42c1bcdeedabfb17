"""MI355X-native ROR-BK (Regularized Orthogonality and Residual based
Block-Kaczmarz, arXiv 2510.02156) behind a C ABI.

``Solver`` wraps one setup handle; ``RorBkFunction`` differentiates a fixed
number of iterations with respect to b and x0.  The raw ``ror_bk_*`` entry
points mirror include/rorbk.h one to one.
"""
from __future__ import annotations

import torch

from .binding import *  # noqa: F401,F403
from .binding import (RORBK_CHECKPOINT, RORBK_PROFILE, RORBK_RECORD, RORBK_REFINE, RORBK_REPLAY,
                      RorBkError, lib, ror_bk_backward, ror_bk_destroy,
                      ror_bk_get_block_inverse, ror_bk_get_form, ror_bk_get_profile,
                      ror_bk_get_record,
                      ror_bk_get_setup, ror_bk_partition,
                      ror_bk_fabgmres, ror_bk_get_sizes, ror_bk_initial_solution,
                      ror_bk_residual, ror_bk_sample, ror_bk_set_proposal,
                      ror_bk_set_refine, ror_bk_set_replay, ror_bk_setup, ror_bk_solve,
                      ror_bk_topk)


class Solver:
    """One ROR-BK setup on the GPU (Algorithm 1, first four steps).

    Dense: ``Solver(A, block_rows, lam)`` with A a 2-D CUDA tensor (float64,
    float32 or bfloat16; ``A64`` the FP64 master for refinement).  CSR:
    ``Solver(None, block_rows, lam, rowptr=, colidx=, values=, shape=)``.
    The tensors must stay alive and unchanged while the solver is used.
    """

    def __init__(self, A=None, block_rows: int = 1, lam: float = 0.0, *, rowptr=None,
                 colidx=None, values=None, shape=None, A64=None, stream=None):
        self._keep = (A, rowptr, colidx, values, A64)
        self.h, self.desc = ror_bk_setup(A, block_rows, lam, stream, rowptr=rowptr,
                                         colidx=colidx, values=values, shape=shape, A64=A64)
        self.k, self.K, self.bmax = ror_bk_get_sizes(self.h)
        self.m, self.n = self.desc.m, self.desc.n
        self.dtype = self.desc.dtype
        self._b_keep = None
        # every solve on the handle replaces its record; backward checks that
        # the record it differentiates is still the one its forward made
        self.generation = 0

    # vector dtype of plain solves on this storage
    def vec_dtype(self, refine: bool = False):
        return torch.float64 if (refine or self.dtype == 0) else torch.float32

    def solve(self, b, x=None, *, seed: int = 0, tol: float = 1e-8, max_iters: int = 1000,
              start_iter: int = 0, refine: bool = False, record: bool = False,
              replay: bool = False, checkpoint_every: int = 0, profile: bool = False):
        """Run ROR-BK from x (zeros if None; updated in place).  Returns (x, info)."""
        vt = self.vec_dtype(refine)
        if x is None:
            x = torch.zeros(self.n, dtype=vt, device=b.device)
        if b.dtype != vt or x.dtype != vt:
            raise TypeError(f"b and x must be {vt} for this solve")
        flags = (RORBK_REFINE if refine else 0) | (RORBK_RECORD if record else 0) | \
                (RORBK_REPLAY if replay else 0) | (RORBK_CHECKPOINT if checkpoint_every else 0) | \
                (RORBK_PROFILE if profile else 0)
        self._b_keep = b
        self.generation += 1
        info = ror_bk_solve(self.h, b, x, seed, tol, max_iters, start_iter, flags,
                            checkpoint_every)
        return x, info

    def backward(self, grad_x):
        """dL/db and dL/dx0 of the last recorded solve, given dL/dx_final."""
        gb = torch.empty(self.m, dtype=grad_x.dtype, device=grad_x.device)
        gx0 = torch.empty(self.n, dtype=grad_x.dtype, device=grad_x.device)
        ror_bk_backward(self.h, grad_x.contiguous(), gb, gx0)
        return gb, gx0

    def setup_arrays(self) -> dict:
        return ror_bk_get_setup(self.h)

    def set_proposal(self, W):
        ror_bk_set_proposal(self.h, W)

    @property
    def column_form(self) -> bool:
        """True if setup chose the column form (n x n stored inverses)."""
        return ror_bk_get_form(self.h) == 1

    def block_inverse(self, t: int):
        """Stored inverse of block t: (A_t A_t^T + lambda I)^{-1} (row form) or
        (A_t^T A_t + lambda I)^{-1} (column form)."""
        if self.column_form:
            return ror_bk_get_block_inverse(self.h, t, self.n)
        off = self.setup_arrays()["offsets"]
        return ror_bk_get_block_inverse(self.h, t, int(off[t + 1] - off[t]))

    def sample(self, seed: int, j0: int, count: int):
        return ror_bk_sample(self.h, seed, j0, count)

    def topk(self, r):
        idx = torch.empty(self.K, dtype=torch.int32, device=r.device)
        ror_bk_topk(self.h, r, idx)
        return idx

    def residual(self, b, x, use_f64_master: bool = False):
        r = torch.empty(self.m, dtype=b.dtype, device=b.device)
        bn = torch.empty(self.k, dtype=torch.float64, device=b.device)
        rrn = ror_bk_residual(self.h, b, x, r, bn, use_f64_master)
        return r, bn, rrn

    def fabgmres(self, b, x=None, *, seed: int = 0, tol: float = 1e-8, max_outer: int = 20,
                 inner_iters: int = 10, eta: float = 1e-1):
        """Flexible AB-GMRES with ROR-BK inner iterations (FP64 storage) from x
        (zeros if None; updated in place).  Returns (x, info)."""
        if x is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=b.device)
        if b.dtype != torch.float64 or x.dtype != torch.float64:
            raise TypeError("flexible AB-GMRES works on double vectors")
        self.generation += 1
        info = ror_bk_fabgmres(self.h, b, x, seed, tol, max_outer, inner_iters, eta)
        return x, info

    def initial_solution(self, b):
        """Algorithm 2's starting iterate for b (same vector type as b);
        returns (x0, coefficient)."""
        x0 = torch.empty(self.n, dtype=b.dtype, device=b.device)
        coef = ror_bk_initial_solution(self.h, b, x0)
        return x0, coef

    def profile(self) -> dict:
        return ror_bk_get_profile(self.h)

    def record(self) -> dict:
        return ror_bk_get_record(self.h, self.K)

    def set_replay(self, tau, I, iters: int):
        ror_bk_set_replay(self.h, tau, I, iters)

    def set_refine(self, inner_iters: int = 50, eta: float = 1e-4):
        ror_bk_set_refine(self.h, inner_iters, eta)

    def close(self):
        if getattr(self, "h", None):
            ror_bk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RorBkFunction(torch.autograd.Function):
    """x_K = ROR-BK(b, x0) over a fixed number of iterations (tol = 0); the
    backward pass gives dL/db and dL/dx0 through the hand-written adjoint with
    the sampled and greedy selections held fixed.  ``checkpoint_every`` > 0
    keeps only every c-th iterate and recomputes the greedy sets."""

    @staticmethod
    def forward(ctx, b, x0, solver, seed, iters, checkpoint_every=0):
        x = x0.detach().clone()
        bb = b.detach().contiguous()
        solver.solve(bb, x, seed=seed, tol=0.0, max_iters=iters,
                     record=not checkpoint_every, checkpoint_every=checkpoint_every)
        ctx.solver = solver
        ctx.b = bb
        ctx.generation = solver.generation
        return x

    @staticmethod
    def backward(ctx, gx):
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError(
                "RorBkFunction.backward: the solver ran another solve after this forward, "
                "so its record belongs to a different run; give each differentiated "
                "forward its own Solver, or run its backward before the next solve")
        gb, gx0 = ctx.solver.backward(gx.contiguous())
        return gb, gx0, None, None, None, None
