"""Differentiable capacitance for torch.autograd, on top of the C ABI.

Two maps, each with a hand-written backward that runs in the library's kernels:

* ``capacitance_eps``: C(eps) -> the m x m capacitance matrix as a function of the
  relative permittivities of dielectric blocks.  The matrix of eq. (4) depends on eps
  only through the jump term of eq. (7) on dielectric panels and through the
  free-charge weights of eq. (8); the backward is the adjoint method
  (A^T lambda_i = w_i, one adjoint GMRES solve per conductor through the transposed
  FFT product) assembled on the GPU into dC/d eps_b.
* ``charges_to_capacitance``: rho -> C by the reduction of eq. (8), a linear map whose
  adjoint scatters the cotangent back onto the conductor panels.
"""
import numpy as np
import torch

from . import voxcap


class _CapacitanceEps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_blocks, problem, base_eps, block_of_voxel, solve_kw):
        eps = np.array(base_eps, dtype=np.float64, copy=True)
        e = eps_blocks.detach().to("cpu", torch.float64).numpy()
        nb = len(e)
        for b in range(nb):
            eps[block_of_voxel == b] = e[b]
        # only the eq. (7) jump terms and eq. (8) weights depend on eps: the problem's
        # setup (spectra, preconditioner blocks) is reused
        problem.update_eps(eps)
        if ctx.needs_input_grad[0]:
            dC, Cm, st = problem.capacitance_grad_eps(block_of_voxel, nb, **solve_kw)
            ctx.save_for_backward(torch.from_numpy(dC))
        else:
            Cm, st = problem.capacitance(**solve_kw)
        ctx.stats = st
        return torch.from_numpy(np.ascontiguousarray(Cm)).to(eps_blocks.device)

    @staticmethod
    def backward(ctx, gC):
        (dC,) = ctx.saved_tensors
        # vector-Jacobian product of the (nblocks, m, m) Jacobian with the m x m cotangent
        g = (dC * gC.detach().to("cpu", torch.float64).unsqueeze(0)).sum(dim=(1, 2))
        return g.to(gC.device), None, None, None, None


def capacitance_eps(scene, block_of_voxel, eps_blocks, device=0, setup=None, problem=None, **solve):
    """C (m x m, farads) of `scene` with the voxels of block b (block_of_voxel == b) set
    to relative permittivity eps_blocks[b]; differentiable in eps_blocks.

    problem: a set-up voxcap.Problem of this scene's geometry to reuse (its
    permittivities are overwritten; see problem_for); None sets one up (with the
    keyword options `setup`) for this call alone.
    solve: keyword options of Problem.capacitance (prec, rtol, ...)."""
    blk = np.ascontiguousarray(block_of_voxel, dtype=np.int32)
    if blk.shape != np.shape(scene["cond_id"]):
        raise ValueError("block_of_voxel must have the grid's shape")
    if not torch.is_tensor(eps_blocks):
        eps_blocks = torch.as_tensor(eps_blocks, dtype=torch.float64)
    if problem is None:
        problem = problem_for(scene, device=device, **dict(setup or {}))
    elif problem.shape != blk.shape:
        raise ValueError("problem and scene grids differ")
    return _CapacitanceEps.apply(eps_blocks, problem, scene["eps_r"], blk, dict(solve))


# the autograd Function itself (eps per block -> C, backward by the adjoint solves)
CapacitanceFn = _CapacitanceEps


def problem_for(scene, device=0, **setup):
    """A set-up Problem of `scene` for repeated capacitance_eps calls (one setup, then
    only permittivity updates)."""
    return voxcap.Problem.from_scene(scene, device).setup(**setup)


class _ChargesToC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, problem):
        rho = rho.contiguous()
        if rho.dtype != torch.float64 or not rho.is_cuda or rho.dim() != 2 or rho.shape[1] != problem.N:
            raise ValueError("rho must be a (nrhs, N) float64 cuda tensor")
        nrhs = rho.shape[0]
        C = torch.empty(problem.m, nrhs, dtype=torch.float64, device=rho.device)
        voxcap.vc_charges_to_capacitance(problem._h, rho, C, nrhs, torch.cuda.current_stream(rho.device))
        ctx.problem = problem
        ctx.nrhs = nrhs
        return C

    @staticmethod
    def backward(ctx, gC):
        gC = gC.contiguous().to(torch.float64)
        grho = torch.empty(ctx.nrhs, ctx.problem.N, dtype=torch.float64, device=gC.device)
        voxcap.vc_charges_to_capacitance_adjoint(ctx.problem._h, gC, grho, ctx.nrhs,
                                                 torch.cuda.current_stream(gC.device))
        return grho, None


def charges_to_capacitance(problem, rho):
    """C[i, j] = 4 pi eps0 dv sum over the panels k of conductor i of eps_adj(k) rho[j, k]
    (eq. 8) for charges rho of shape (nrhs, N) on the GPU; differentiable in rho."""
    return _ChargesToC.apply(rho, problem)
