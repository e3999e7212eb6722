"""He-normal network parameters for the CNN + attention + backbone stack.

Shapes follow the network the library evaluates:

* two weight groups, ``diffuse`` (template layers 0-7) and ``highlight``
  (layers 8-11), each with
  conv1 ``w1`` [8,1,3,3,3] + ``b1`` [8], conv2 ``w2`` [16,8,3,3,3] + ``b2`` [16],
  squeeze-excitation ``s1`` [4,16] + ``c1`` [4] and ``s2`` [16,4] + ``c2`` [16];
* the backbone: ``n_linear`` Linear layers, ``A[0]`` [width, 1057],
  ``A[1..n-2]`` [width, width], ``A[n-1]`` [1, width], with biases ``beta[i]``.

Weights are drawn ``standard_normal(shape) * sqrt(2 / fan_in)`` from
``numpy.random.default_rng(seed)`` in the order diffuse w1, w2, s1, s2;
highlight w1, w2, s1, s2; backbone A[0..n-1].  fan_in is in_channels * 27 for a
convolution and in_features for a Linear layer.  Biases are zero unless
``bias_scale`` is given, in which case they are drawn afterwards in the same
group order as ``bias_scale * standard_normal``.
"""

import numpy as np

DESCRIPTOR = 1057          # 12 layers x (80 attention features + 8 squeeze stats) + albedo
GROUP_KEYS = ("w1", "b1", "w2", "b2", "s1", "c1", "s2", "c2")


def _he(rng, shape, fan_in):
    return (rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)).astype(np.float32)


def he_init(width, n_linear, seed=1, bias_scale=0.0, lam=0.6, gamma=4.0):
    """Return the parameter dict described in the module docstring."""
    if n_linear < 2:
        raise ValueError("the backbone needs at least two Linear layers")
    rng = np.random.default_rng(seed)
    groups = {}
    for name in ("diffuse", "highlight"):
        groups[name] = {
            "w1": _he(rng, (8, 1, 3, 3, 3), 27),
            "w2": _he(rng, (16, 8, 3, 3, 3), 216),
            "s1": _he(rng, (4, 16), 16),
            "s2": _he(rng, (16, 4), 4),
        }
    dims = [DESCRIPTOR] + [width] * (n_linear - 1) + [1]
    A = [_he(rng, (dims[i + 1], dims[i]), dims[i]) for i in range(n_linear)]
    zeros = {"b1": 8, "c1": 4, "b2": 16, "c2": 16}
    for name in ("diffuse", "highlight"):
        for k, n in zeros.items():
            groups[name][k] = np.zeros(n, np.float32)
    beta = [np.zeros(dims[i + 1], np.float32) for i in range(n_linear)]
    if bias_scale:
        for name in ("diffuse", "highlight"):
            for k, n in zeros.items():
                groups[name][k] = (bias_scale * rng.standard_normal(n)).astype(np.float32)
        beta = [(bias_scale * rng.standard_normal(dims[i + 1])).astype(np.float32)
                for i in range(n_linear)]
    return {"width": width, "n_linear": n_linear, "lam": float(lam),
            "gamma": float(gamma), "groups": groups, "A": A, "beta": beta}


def zeros_like(params):
    """Same shapes with every weight and bias set to zero."""
    out = {k: params[k] for k in ("width", "n_linear", "lam", "gamma")}
    out["groups"] = {g: {k: np.zeros_like(v) for k, v in d.items()}
                     for g, d in params["groups"].items()}
    out["A"] = [np.zeros_like(a) for a in params["A"]]
    out["beta"] = [np.zeros_like(b) for b in params["beta"]]
    return out


# Point counts of the paper's template layers (8 diffuse sphere layers, 4
# highlight cone layers) and the width of the modules' merges.
TEMPLATE_COUNTS = (6, 8, 12, 16, 24, 32, 48, 48, 32, 16, 16, 8)
MODULE_MERGE = 64


def he_init_modules(seed=2, bias_scale=0.0):
    """Weights of the six layer-by-layer modules and three merges of the
    paper's backbone, He-normal from default_rng(seed), as a list of float32
    arrays in the blob order: for type 0..2 (graded transmittance, density,
    phase), for group 0..1 (diffuse layers 0-7, highlight 8-11), for each
    step k (from each group layer but its last): S1 [2][8], e1 [2], S2 [a][2],
    e2 [a], F1 [b][a], f1 [b], F2 [b][b], f2 [b] with a = n_k + 2 and
    b = n_(k+1); then for type 0..2: M [64][56], mb [64].  Biases are zero
    unless bias_scale is given."""
    rng = np.random.default_rng(seed)
    out = []

    def bias(n):
        return (bias_scale * rng.standard_normal(n)).astype(np.float32) if bias_scale else np.zeros(n, np.float32)

    for _tau in range(3):
        for grp in range(2):
            k0, k1 = (0, 7) if grp == 0 else (8, 11)
            for k in range(k0, k1):
                a, b = TEMPLATE_COUNTS[k] + 2, TEMPLATE_COUNTS[k + 1]
                out += [_he(rng, (2, 8), 8), bias(2), _he(rng, (a, 2), 2), bias(a),
                        _he(rng, (b, a), a), bias(b), _he(rng, (b, b), b), bias(b)]
    cat = TEMPLATE_COUNTS[7] + TEMPLATE_COUNTS[11]
    for _tau in range(3):
        out += [_he(rng, (MODULE_MERGE, cat), cat), bias(MODULE_MERGE)]
    return out
