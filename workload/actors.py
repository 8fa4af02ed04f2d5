"""Seeded actor weights for the K-actor ensemble.

Each actor is an MLP S -> H -> H -> A with tanh after every layer, so the
action mean lies in [-1, 1].  Weights use Xavier-uniform initialisation
(limit sqrt(6 / (fan_in + fan_out))) drawn in float64 from numpy's PCG64 with
seed seed_base + k and cast to float32; biases are zero unless bias_std > 0.

Packed layout (float32, actor-major, each matrix input-major so that a
row-vector input multiplies it from the left):
    for k in 0..K-1: W1[S][H], b1[H], W2[H][H], b2[H], W3[H][A], b3[A]
"""
from __future__ import annotations

import numpy as np

from .configs import ActorConfig


def layer_shapes(cfg: ActorConfig):
    S, H, A = cfg.in_dim, cfg.hidden, cfg.out_dim
    return [("W1", (S, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, A)), ("b3", (A,))]


def params_per_actor(cfg: ActorConfig) -> int:
    return sum(int(np.prod(s)) for _, s in layer_shapes(cfg))


def make_actor_weights(cfg: ActorConfig):
    """List of K dicts {W1,b1,W2,b2,W3,b3} of float32 arrays."""
    actors = []
    for k in range(cfg.n_actors):
        rng = np.random.default_rng(cfg.seed_base + k)
        p = {}
        for name, shape in layer_shapes(cfg):
            if name.startswith("W"):
                lim = np.sqrt(6.0 / (shape[0] + shape[1]))
                p[name] = rng.uniform(-lim, lim, size=shape).astype(np.float32)
            else:
                if cfg.bias_std > 0:
                    p[name] = (cfg.bias_std * rng.standard_normal(shape)).astype(np.float32)
                else:
                    p[name] = np.zeros(shape, dtype=np.float32)
        actors.append(p)
    return actors


def pack_actor_weights(actors) -> np.ndarray:
    """Concatenate K actors into the flat float32 layout described above."""
    parts = []
    for p in actors:
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            parts.append(np.ascontiguousarray(p[name], dtype=np.float32).ravel())
    return np.concatenate(parts)


def unpack_actor_weights(flat: np.ndarray, cfg: ActorConfig):
    flat = np.asarray(flat, dtype=np.float32).ravel()
    out, off = [], 0
    for _ in range(cfg.n_actors):
        p = {}
        for name, shape in layer_shapes(cfg):
            n = int(np.prod(shape))
            p[name] = flat[off:off + n].reshape(shape).copy()
            off += n
        out.append(p)
    if off != flat.size:
        raise ValueError(f"packed weights have {flat.size} floats, expected {off}")
    return out
