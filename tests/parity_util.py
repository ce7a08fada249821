"""Shared helpers of the GPU parity tests: per-variable error norms (R24's
"rel": the 2-norm over all blocks, cells and snapshots, per conserved
variable) and the FP64 rounding floor of the residual on a given state."""
import torch

from oracle import hb_oracle as O


def per_var_errors(blocks, x, ref):
    """[||x_v - ref_v|| / ||ref_v|| for v in 0..3] over all blocks, cells and
    snapshots."""
    xs, rs = O.split(blocks, x), O.split(blocks, ref)
    out = []
    for v in range(4):
        num = sum(float(((a[:, v] - b[:, v]) ** 2).sum()) for a, b in zip(xs, rs))
        den = sum(float((b[:, v] ** 2).sum()) for b in rs)
        out.append((num / den) ** 0.5 if den > 0 else num ** 0.5)
    return out


def per_var_rel(blocks, x, ref):
    return max(per_var_errors(blocks, x, ref))


def fp64_floor(blocks, q, flow, solver, cuts=(), seed=5):
    """Per variable, the relative change of the oracle's FP64 residual when
    every node coordinate and every state value is perturbed by one unit in
    the last place (random sign): the spread that rounding alone puts
    between two correct FP64 evaluations that order their operations
    differently.  Where the residual is small against the face fluxes that
    form it (near convergence, thin wall cells), this floor exceeds the
    1e-12 FP64 tolerance."""
    g = torch.Generator().manual_seed(seed)
    eps = 2.0 ** -53

    def sign(shape):
        return torch.randint(0, 2, shape, generator=g).to(torch.float64) * 2 - 1

    r0 = O.residual_all(blocks, q, flow, solver, cuts)
    xys = [b.xy * (1 + eps * sign(b.xy.shape)) for b in blocks]
    rx = O.residual_all(blocks, q, flow, solver, cuts, None, xys)
    rq = O.residual_all(blocks, q * (1 + eps * sign(q.shape)), flow, solver, cuts)
    ex, eq = per_var_errors(blocks, rx, r0), per_var_errors(blocks, rq, r0)
    return [max(a, b) for a, b in zip(ex, eq)], r0


def fp64_tolerance(floor, factor=4.0):
    """The FP64 residual tolerance per variable: 1e-12, or a few times the
    rounding floor where that is larger."""
    return [max(1e-12, factor * f) for f in floor]


def block_trajectory(args):
    """Oracle iterations of one block on its own (blocks without cuts are
    independent): returns (states after each iteration count in `marks`,
    per-iteration sums over the block's cells and snapshots of (R*_rho/V)^2).
    Runs in a worker process; args = (problem name, block index, marks,
    threads)."""
    from paper_1304_7654_amd import synth
    name, k, marks, threads = args
    torch.set_num_threads(threads)
    p = synth.make_problem(name)
    blocks, flow, solver = O.from_synth(p)
    q = O.split(blocks, torch.as_tensor(synth.initial_state(p)))[k].reshape(-1).clone()
    b = blocks[k]
    cs = b.ns * b.ni * b.nj
    states, sums, done = {}, [], 0
    for m in marks:
        q, nr = O.rk_iterate([b], q, flow, solver, m - done)
        sums.append(nr ** 2 * cs)
        states[m] = q.clone()
        done = m
    return states, torch.cat(sums)
