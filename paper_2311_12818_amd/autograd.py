"""Differentiable manifold walks: a ``torch.autograd.Function`` whose forward
is the batched walk (manifold_walk_batch + manifold_walk_fp64) and whose
backward is manifold_walk_adjoint, the implicit-function-theorem adjoint of
the converged chains (Sec. 5.2).

Differentiable inputs are the shading points x_D [3, N], the light points
x_L [3, N] and the height-field parameters theta [P] (amplitude, phase per
sine).  Outputs are the converged vertices [3, K, N], the generalized geometry
term G [N] and the walk status [N] (not differentiable).  Chains that do not
converge have zero gradients.  A change of theta updates the device scene in
place (mpg_scene_set_params: vertices, normals, BVH refit, area tables).
"""
from __future__ import annotations

from . import (FORM_PERSISTENT, MPGError, Endpoints, Scene, Workspace, empty_chains, manifold_walk_adjoint,
               manifold_walk_batch, manifold_walk_fp64, walk_outputs)


class WalkProblem:
    """What a differentiable walk keeps fixed: the device scene (its
    height-field parameters follow theta through mpg_scene_set_params), the
    walk parameters, the shading normals, lengths, types and p_0 objects of
    the chains, and the seed chains every forward starts from."""

    def __init__(self, scene: Scene, params, nD, length, types, obj1, seed_prim, seed_pos, seed_status=None):
        self._scene = scene
        # the persistent form needs a workspace for the walk and the adjoint
        self.ws = Workspace(int(length.shape[0])) if params.form == FORM_PERSISTENT else None
        self.params = params
        self.nD, self.length, self.types, self.obj1 = nD, length, types, obj1
        self.seed_prim, self.seed_pos, self.seed_status = seed_prim, seed_pos, seed_status
        self._theta = None

    def scene(self, theta) -> Scene:
        if theta.numel() != self._scene.n_params:
            raise MPGError(f"theta has {theta.numel()} entries, the scene has {self._scene.n_params} parameters")
        th = theta.detach().float()
        if self._theta is None or not bool((th == self._theta).all()):
            self._scene.set_params(th)
            self._theta = th.clone()
        return self._scene

    def endpoints(self, xD, xL) -> Endpoints:
        return Endpoints.from_tensors(xD.detach().float(), self.nD, xL.detach().float(), self.length, self.types,
                                      self.obj1)


def _torch():
    import torch
    return torch


def _function():
    torch = _torch()

    class ManifoldWalk(torch.autograd.Function):
        @staticmethod
        def forward(ctx, xD, xL, theta, problem: WalkProblem):
            scene = problem.scene(theta)
            ep = problem.endpoints(xD, xL)
            prm = problem.params
            prim, pos = empty_chains(ep.N, xD.device)
            outs = walk_outputs(ep.N, xD.device)
            manifold_walk_batch(scene, prm, ep, problem.seed_prim, problem.seed_pos, problem.seed_status,
                                out_prim=prim, out_pos=pos, outs=outs, ws=problem.ws)
            manifold_walk_fp64(scene, prm, ep, prim, pos, outs)
            ctx.problem, ctx.ep = problem, ep
            ctx.theta_value = theta.detach().clone()
            ctx.theta_meta = (theta.shape, theta.dtype)
            ctx.xD_dtype, ctx.xL_dtype = xD.dtype, xL.dtype
            ctx.save_for_backward(prim, pos, outs["status"])
            status = outs["status"]
            ctx.mark_non_differentiable(status)
            return pos, outs["G"], status

        @staticmethod
        def backward(ctx, grad_pos, grad_G, _grad_status):
            prim, pos, status = ctx.saved_tensors
            # the scene may have moved to another theta since this forward
            scene, ep = ctx.problem.scene(ctx.theta_value), ctx.ep
            gp = None if grad_pos is None else grad_pos.float().contiguous()
            gG = None if grad_G is None else grad_G.float().contiguous()
            dev = pos.device
            gth = torch.zeros(max(1, scene.n_params), dtype=torch.float32, device=dev)
            gxD, gxL, gth = manifold_walk_adjoint(scene, ctx.problem.params, ep, prim, pos, status, gp, gG,
                                                  grad_theta=gth, ws=ctx.problem.ws)
            shape, dtype = ctx.theta_meta
            g_theta = gth[:scene.n_params].to(dtype).reshape(shape) if ctx.needs_input_grad[2] else None
            return (gxD.to(ctx.xD_dtype) if ctx.needs_input_grad[0] else None,
                    gxL.to(ctx.xL_dtype) if ctx.needs_input_grad[1] else None, g_theta, None)

    return ManifoldWalk


_FN = None


def manifold_walk(xD, xL, theta, problem: WalkProblem):
    """Differentiable batched walk: returns (pos [3, K, N], G [N], status [N])."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(xD, xL, theta, problem)
