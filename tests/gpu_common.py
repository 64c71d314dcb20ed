"""Shared helpers of the GPU parity tests: tolerances and context builders.

The tolerances are the ones the path is held to: FP32 forward outputs within
1e-5 relative (plus a 1e-7 absolute floor), gradients within 1e-4 relative
norm-wise, and per entry within 1e-4 of the entry plus 1e-4 of its
magnitude (from the oracle: the same backward pass run on absolute values of
every weight, activation and adjoint).  Rounding error of a computed entry is
relative to that magnitude, not to the possibly cancelled value: a sum of n
FP32 terms in any order is off by at most about n u sum|term_k| (u = 2^-24),
typically sqrt(n) u sum|term_k|; 1e-4 is about 1700 u.  Where an entry
depends on a discrete decision (ReLU branch, density clamp, depth-error sign)
that lies within 1e-5 relative of its tie, FP32 and FP64 may both be right
and disagree: such entries may further differ by the oracle's allowance (the
tie samples' contributions with every branch taken); everything else must
match to the bound above, and the norm-wise bound is taken over the entries
that no such decision reaches.
"""
import numpy as np

import oracle
import paper_2304_05735_amd as pk


def assert_fwd_close(gpu, ref, rtol=1e-5, atol=1e-7, what=""):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(gpu - ref)
    bad = err > rtol * np.abs(ref) + atol
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), gpu[bad][:5], ref[bad][:5])
    return float(err.max())


def assert_grad_close(gpu, ref, mass, allow=None, rtol=1e-4, mtol=1e-4, what=""):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    mass = np.asarray(mass, np.float64)
    allow = np.zeros_like(ref) if allow is None else np.asarray(allow, np.float64)
    d = gpu - ref
    nr = np.linalg.norm(ref)
    # norm-wise over the entries no tied decision reaches (those are bounded
    # one by one below, by their allowance)
    clean = allow == 0
    assert np.linalg.norm(d[clean]) <= rtol * nr + 1e-30, (
        what, np.linalg.norm(d[clean]) / max(nr, 1e-30))
    bad = np.abs(d) > rtol * np.abs(ref) + mtol * mass + allow
    assert not bad.any(), (what, int(bad.sum()), float(np.abs(d).max()), np.flatnonzero(bad)[:5])
    return float(np.linalg.norm(d) / max(nr, 1e-30))


def make_pair(L, nmin, nmax, log2T, N, B, frames, box, precision=pk.PREC_FP32, mlp_layers=1,
              **kw):
    """A GPU context and an oracle context holding the same object and keyframes."""
    cfg = pk.default_config(n_levels=L, base_res=nmin, max_res=nmax, log2_table_size=log2T,
                            samples_per_ray=N, rays_per_step=B, autotune=0,
                            precision=precision, mlp_layers=mlp_layers, **kw)
    g = pk.Context(cfg)
    ocfg = oracle.make_config(L=L, nmin=nmin, nmax=nmax, log2T=log2T, N=N,
                              lambda_depth=float(cfg.lambda_depth),
                              lambda_density=float(cfg.lambda_density), lr=float(cfg.lr),
                              beta1=float(cfg.beta1), beta2=float(cfg.beta2), eps=float(cfg.eps))
    o = oracle.OracleContext(ocfg, mlp_layers=mlp_layers)
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
