"""Helpers for the GPU tests: run the HIP path through the C-ABI binding and
compute oracle references.  Imported only by tests."""
import numpy as np
import torch

from oracle import dtm as odtm

TOL_F64 = 1e-9  # L1(pi) against the float64 oracle, float64 path
TOL_F32 = 1e-6  # L1(pi) against the float64 oracle, float32 path


def lib():
    from paper_2509_20500_amd import dtm
    dtm.lib()  # fails loudly when the HIP library is missing
    return dtm


def tdtype(dt):
    return torch.float32 if dt == "f32" else torch.float64


def oracle_pi(scene):
    return odtm.stationary_solve(odtm.transition_matrix(scene))


def default_opts(dt):
    """Stop rule targets: 1e-6 for float32, 1e-10 for float64 (so that the
    float64 path lands well inside its 1e-9 parity bar)."""
    d = lib()
    return d.opts(tol=1e-6) if dt == "f32" else d.opts(tol=1e-10)


def run_batched(scenes, dt, x0=None, solve_opts=None, tiles=None, return_plan=False):
    d = lib()
    if solve_opts is None:
        solve_opts = default_opts(dt)
    plan = d.Plan(scenes, dt, solve_opts, tiles)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=tdtype(dt), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve(pi, infos, x0)
    torch.cuda.synchronize()
    out = pi.cpu().numpy().astype(np.float64), d.infos_to_numpy(infos), plan.pi_offsets
    if return_plan:
        return out + (plan, ws)
    plan.close()
    return out


def split(packed, offsets):
    return [packed[offsets[p]:offsets[p + 1]] for p in range(len(offsets) - 1)]
