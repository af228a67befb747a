"""Seeded random model weights in the documented manifest order.

A model's weights travel as one flat float64 vector.  The manifest (the order
and shape of every tensor in it) is part of the interface and is written out
in ``include/nnp.h``; this module only lists the shapes so that it can draw
Xavier-normal matrices (std = sqrt(2 / (fan_in + fan_out))) and Gaussian
biases in that order.  Matrices are stored row-major as [out][in].
"""

from dataclasses import dataclass

import numpy as np

N_SPECIES = 4


@dataclass(frozen=True)
class ModelSpec:
    kind: str            # "cons" or "nc"
    width: int           # F (cons) or F' (nc)
    n_layers: int        # message-passing layers (nc: 1)
    n_rbf: int           # Bessel functions of the embedding filter
    cutoff: float        # Angstrom
    n_species: int = N_SPECIES
    n_s: int = 8         # nc scalar heads
    n_l: int = 2         # nc vector heads
    n_c: int = 8         # nc query/key dimension
    poly_p: int = 5      # nc polynomial envelope order


CONS_CFG0 = ModelSpec("cons", 32, 2, 16, 5.0)
CONS_CFG1 = ModelSpec("cons", 128, 3, 16, 5.0)
NC_CFG0 = ModelSpec("nc", 16, 1, 8, 3.5)
NC_CFG1 = ModelSpec("nc", 32, 1, 8, 3.5)


def _block(prefix, F, K):
    return [
        (prefix + "W1", (F, F), "w"), (prefix + "b1", (F,), "b"),
        (prefix + "W2", (3 * F, F), "w"), (prefix + "b2", (3 * F,), "b"),
        (prefix + "Wr", (3 * F, K), "w"), (prefix + "br", (3 * F,), "b"),
        (prefix + "U", (F, F), "w"), (prefix + "V", (F, F), "w"),
        (prefix + "M1", (F, 2 * F), "w"), (prefix + "m1", (F,), "b"),
        (prefix + "M2", (3 * F, F), "w"), (prefix + "m2", (3 * F,), "b"),
    ]


def cons_manifest(spec):
    F, K = spec.width, spec.n_rbf
    ent = [("emb", (spec.n_species, F), "w")]
    for layer in range(spec.n_layers):
        ent += _block(f"l{layer}.", F, K)
    ent += [("Wo", (F, F), "w"), ("bo", (F,), "b"), ("wo", (1, F), "w"),
            ("beta", (spec.n_species,), "b")]
    return ent


def nc_manifest(spec):
    F, K = spec.width, spec.n_rbf
    H = spec.n_s + spec.n_l
    ent = [("emb", (spec.n_species, F), "w")]
    ent += _block("l0.", F, K)
    ent += [("Wq", (H, spec.n_c, F), "w"), ("Wk", (H, spec.n_c, F), "w"),
            ("WV", (spec.n_l, F), "w")]
    return ent


def manifest(spec):
    return cons_manifest(spec) if spec.kind == "cons" else nc_manifest(spec)


def manifest_size(spec):
    return int(sum(int(np.prod(s)) for _, s, _ in manifest(spec)))


def random_weights(spec, seed, bias_std=0.1, weight_gain=1.0):
    """Flat float64 weight vector: Xavier-normal matrices, N(0, bias_std^2)
    biases, in manifest order."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, shape, kind in manifest(spec):
        if kind == "w":
            fan_out, fan_in = shape[-2], shape[-1]
            std = weight_gain * np.sqrt(2.0 / (fan_in + fan_out))
            parts.append(rng.normal(scale=std, size=shape).ravel())
        else:
            parts.append(rng.normal(scale=bias_std, size=shape).ravel() if bias_std > 0
                         else np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float64)
