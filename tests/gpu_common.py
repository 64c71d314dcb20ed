"""Shared helpers of the GPU parity tests: tolerances and context builders.

The tolerances are the ones the path is held to: FP32 forward outputs within
1e-5 relative (plus a 1e-7 absolute floor); gradients within 1e-4 relative
norm-wise per tensor (the grid, W1, each hidden-to-hidden matrix, W2, W3,
W4), and per entry within 1e-4 of the entry plus 1e-4 of its magnitude
(from the oracle: the same backward pass run on absolute values of every
weight, activation and adjoint).  Rounding error of a computed entry is
relative to that magnitude, not to the possibly cancelled value: a sum of n
FP32 terms in any order is off by at most about n u sum|term_k| (u = 2^-24),
typically sqrt(n) u sum|term_k|; 1e-4 is about 1700 u.

Where a decision (a ReLU branch, the density clamp, the depth-error sign)
lies within 1e-5 relative of its tie, FP32 and FP64 may both be right and
take different branches.  The oracle's allowance holds, per entry, the change
that the other branch of each such decision makes (to first order: the
forward stays, one adjoint is switched on or off at the tied unit and carried
down).  Entries may differ by their allowance on top of the bound above, and
the norm-wise bound applies to what exceeds the allowance.  The allowance is
reported per tensor (share of entries that carry one, its norm against the
tensor's) and its norm is capped, so it cannot swallow the comparison.
"""
import numpy as np

import oracle
import paper_2304_05735_amd as pk

# allowance norm / gradient norm, per tensor: FP32 ties stay below 1e-2 of a
# tensor (measured 2e-4 ... 6e-3); BF16 widens the ties by what upstream BF16
# decisions can move a pre-activation
ALLOW_CAP_FP32 = 0.02
ALLOW_CAP_BF16 = 0.3


def assert_fwd_close(gpu, ref, rtol=1e-5, atol=1e-7, what=""):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(gpu - ref)
    bad = err > rtol * np.abs(ref) + atol
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), gpu[bad][:5], ref[bad][:5])
    return float(err.max())


def tensor_cuts(o, oid):
    """(name, begin, end) of every tensor in the parameter vector of an oracle
    object: the grid, W1, the hidden-to-hidden matrices, W2, W3, W4."""
    ob = o.objects[oid]
    pg = oracle.grid_params(ob.lv)
    din = 2 * ob.lv.L
    sizes = [("grid", pg), ("W1", 64 * din)]
    sizes += [(f"Wh{k}", 64 * 64) for k in range(1, o.mlp_layers)]
    sizes += [("W2", 16 * 64), ("W3", 64 * 15), ("W4", 3 * 64)]
    cuts, at = [], 0
    for name, n in sizes:
        cuts.append((name, at, at + n))
        at += n
    assert at == o.n_params(oid)
    return cuts


def assert_grad_close(gpu, ref, mass, allow=None, rtol=1e-4, mtol=1e-4, what="", cuts=None,
                      extra=None, norm_tol=None, cap=ALLOW_CAP_FP32, verbose=True):
    """Per entry: |gpu - ref| <= rtol |ref| + mtol mass + allow (+ extra, a
    further per-entry allowance, e.g. of BF16 rounding decisions).  Per
    tensor: the norm of what exceeds the allowance is at most norm_tol[name]
    (default rtol) times the tensor's norm, and the allowance's norm at most
    cap times it.  Returns the largest norm-wise relative error of a tensor."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    mass = np.asarray(mass, np.float64)
    allow = np.zeros_like(ref) if allow is None else np.asarray(allow, np.float64)
    extra = np.zeros_like(ref) if extra is None else np.asarray(extra, np.float64)
    d = gpu - ref
    bad = np.abs(d) > rtol * np.abs(ref) + mtol * mass + allow + extra
    if cuts is None:
        cuts = [("all", 0, ref.size)]
    if bad.any():
        rows = []
        for j in np.flatnonzero(bad)[:12]:
            name, a, _ = next(c for c in cuts if c[1] <= j < c[2])
            rows.append(f"{name}[{j - a}] gpu {gpu[j]:.6e} ref {ref[j]:.6e} mass {mass[j]:.3e} "
                        f"allow {allow[j]:.3e} extra {extra[j]:.3e}")
        print(f"  {what}: {int(bad.sum())} entries beyond the bound:\n    " + "\n    ".join(rows),
              flush=True)
    assert not bad.any(), (what, int(bad.sum()), float(np.abs(d).max()), np.flatnonzero(bad)[:5])
    worst, rows = 0.0, []
    for name, a, b in cuts:
        nr = np.linalg.norm(ref[a:b])
        if nr == 0.0:
            assert not d[a:b].any(), (what, name)
            continue
        excess = np.maximum(np.abs(d[a:b]) - allow[a:b], 0.0)
        rel = float(np.linalg.norm(d[a:b]) / nr)
        rex = float(np.linalg.norm(excess) / nr)
        ral = float(np.linalg.norm(allow[a:b]) / nr)
        share = float(np.mean(allow[a:b] > 0))
        tol = rtol if norm_tol is None else norm_tol.get(name, rtol)
        rows.append(f"{name} {rel:.1e} (beyond allowance {rex:.1e} <= {tol:.1e}; "
                    f"allowance on {share:.3f} of entries, norm {ral:.1e})")
        assert rex <= tol, (what, name, rex, tol)
        assert ral <= cap, (what, name, "allowance norm", ral, cap)
        worst = max(worst, rel)
    if verbose:
        print(f"  {what}: " + "; ".join(rows), flush=True)
    return worst


def make_pair(L, nmin, nmax, log2T, N, B, frames, box, precision=pk.PREC_FP32, mlp_layers=1,
              bf16_oracle=False, **kw):
    """A GPU context and an oracle context holding the same object and keyframes
    (bf16_oracle: the oracle's BF16 mode of the MLP)."""
    cfg = pk.default_config(n_levels=L, base_res=nmin, max_res=nmax, log2_table_size=log2T,
                            samples_per_ray=N, rays_per_step=B, precision=precision,
                            mlp_layers=mlp_layers, **{"autotune": 0, **kw})
    g = pk.Context(cfg)
    ocfg = oracle.make_config(L=L, nmin=nmin, nmax=nmax, log2T=log2T, N=N,
                              lambda_depth=float(cfg.lambda_depth),
                              lambda_density=float(cfg.lambda_density), lr=float(cfg.lr),
                              beta1=float(cfg.beta1), beta2=float(cfg.beta2), eps=float(cfg.eps))
    o = oracle.OracleContext(ocfg, mlp_layers=mlp_layers, bf16=bf16_oracle)
    gid = g.add_object(box["instance"], box["t"], box["yaw"], box["half"])
    oid = o.add_object(box["instance"], box["t"], box["yaw"], box["half"])
    assert gid == oid
    for cam, rgb, mask, depth in frames:
        _, na = g.add_keyframe(cam, rgb, mask, depth)
        nb = o.add_keyframe(cam, rgb, mask, depth)
        assert na == nb
    return g, o, gid


def oracle_grad(o, oid, step, B, **kw):
    """Oracle loss, gradient, magnitude and tie allowance of one step."""
    P = o.n_params(oid)
    mass, allow = np.zeros(P), np.zeros(P)
    loss, g, rays = o.loss_and_grad(oid, step, B, mass=mass, ambiguous=allow, **kw)
    return loss, g, mass, allow, rays


def bf16_reference(o, oid, step, B, seeds=(1, 2, 3), jitter=3e-6):
    """The oracle's BF16-mode step for a GPU BF16 comparison: loss, gradient,
    magnitude, tie allowance, the bound of the BF16 rounding decisions per
    entry and for the loss, and per tensor the spread of the gradient under
    operand perturbations of FP32 size: the largest norm-wise change that
    moving every rounded operand by up to `jitter` of itself makes (three
    deterministic perturbations).  A BF16 value within FP32 error of a
    rounding midpoint may round either way on the GPU; this spread measures
    how far such other choices move each tensor, the loose per-entry bound
    how far they can move each entry at most."""
    assert o.bf16
    P = o.n_params(oid)
    mass, allow, bam, la = np.zeros(P), np.zeros(P), np.zeros(P), np.zeros(1)
    loss, g, rays = o.loss_and_grad(oid, step, B, mass=mass, ambiguous=allow, bf16_allow=bam,
                                    loss_allow=la)
    cuts = tensor_cuts(o, oid)
    spread = {name: 0.0 for name, _, _ in cuts}
    lspread = 0.0
    try:
        oracle.set_bf16_jitter(jitter)
        for sd in seeds:
            oracle.set_jitter_seed(sd)
            lj, gj, _ = o.loss_and_grad(oid, step, B)
            lspread = max(lspread, abs(lj - loss))
            for name, a, b in cuts:
                nr = np.linalg.norm(g[a:b])
                if nr > 0:
                    spread[name] = max(spread[name], float(np.linalg.norm(gj[a:b] - g[a:b]) / nr))
    finally:
        oracle.set_bf16_jitter(0.0)
        oracle.set_jitter_seed(0)
    return dict(loss=loss, grad=g, mass=mass, allow=allow, bf16_allow=bam, loss_allow=float(la[0]),
                spread=spread, loss_spread=lspread, cuts=cuts, rays=rays)


def assert_bf16_close(gl, gg, ref, what="", k=3.0):
    """GPU BF16 step against the oracle's BF16 mode (bf16_reference).  Loss:
    within 1e-5 relative plus k times its perturbation spread, and within the
    rigorous bound of the BF16 decisions.  Gradient: per entry within the
    FP32 bound plus the tie allowance plus the rigorous bound of the BF16
    decisions; per tensor, beyond the tie allowance, within 1e-4 plus k
    times the tensor's perturbation spread."""
    ol = ref["loss"]
    lerr = abs(gl - ol)
    ltol = 1e-5 * abs(ol) + k * ref["loss_spread"]
    print(f"  {what}: loss {gl:.7f} vs BF16 oracle {ol:.7f}: |diff| {lerr:.2e} <= {ltol:.2e} "
          f"(rigorous bound {ref['loss_allow']:.2e})", flush=True)
    assert lerr <= ltol, (what, "loss", lerr, ltol)
    assert lerr <= 1e-5 * abs(ol) + ref["loss_allow"], (what, "loss bound")
    norm_tol = {name: 1e-4 + k * s for name, s in ref["spread"].items()}
    return assert_grad_close(gg, ref["grad"], ref["mass"], ref["allow"], what=what,
                             cuts=ref["cuts"], extra=ref["bf16_allow"], norm_tol=norm_tol,
                             cap=ALLOW_CAP_BF16)
