"""CPU reference for the learned schedule (test infrastructure only).

The learned schedule is not part of the paper's method: a small network
predicts each candidate pair's search cost so that the narrow phase can take
the costliest pairs first.  It only reorders pairs, so nothing here decides a
result; this module is the plain float64 reference the GPU features, network
and gradients are checked against.

Network (kept in this one place on the CPU side):
    x  = bf16((feat - mean) * istd)            (normalization in float32)
    z1 = x W1q + b1,  h1 = relu(z1)
    z2 = h1 W2q + b2, h2 = relu(z2)
    y  = h2 . w3 + b3
with W1q, W2q the bf16-rounded weights (the values the matrix cores see).
`forward(..., round_h1=True)` also rounds h1 to bf16 as the GPU does before
its second product; the gradient reference differentiates the smooth network
(round_h1=False), the function whose gradient the GPU approximates.

Parameter vector layout: W1[16][64], b1[64], W2[64][64], b2[64], W3[64], b3.
"""
import numpy as np

from . import eps as _eps, eval_F as _eval_F, levels_needed as _levels

NF, H = 16, 64
SIZES = [("W1", (NF, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params):
    params = np.asarray(params, np.float64).reshape(-1)
    assert params.size == N_PARAMS
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = params[off:off + k].reshape(shape)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SIZES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def normalize(feat, norm):
    """The network input: bf16 of the float32-normalized features."""
    feat = np.asarray(feat, np.float32).reshape(-1, NF)
    norm = np.asarray(norm, np.float32).reshape(2, NF)
    return bf16((feat - norm[0]) * norm[1])


def quantized(params):
    """Parameters with the two weight matrices rounded to bf16 (biases and w3 stay float32)."""
    p = unpack(np.asarray(params, np.float32).astype(np.float64))
    p["W1"] = bf16(p["W1"])
    p["W2"] = bf16(p["W2"])
    return pack(p)


def forward(params, x, round_h1=False):
    """y for network input x (n x 16, already normalized); params used as given (float64)."""
    p = unpack(params)
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    if round_h1:
        h1 = bf16(h1)
    z2 = h1 @ p["W2"] + p["b2"]
    return np.maximum(z2, 0.0) @ p["w3"] + p["b3"][0]


def loss(params, x, label):
    """Mean squared error of the predictions."""
    e = forward(params, x) - np.asarray(label, np.float64)
    return float(np.mean(e * e))


def grad(params, x, label):
    """Gradient of `loss` with respect to the parameter vector (backpropagation by hand)."""
    p = unpack(params)
    label = np.asarray(label, np.float64)
    n = x.shape[0]
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    dy = 2.0 * (y - label) / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(0)
    return pack(g)


def adam(params, g, m, v, step, lr, beta1, beta2, eps):
    """One Adam step (bias-corrected moments), all float64."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Scheduling features of one query (4 points at t = 0 then at t = 1).
# ---------------------------------------------------------------------------
def _log_ratio(x, delta):
    return np.float32(np.log2(1.0 + abs(x) / delta))


def _bounds(kind, q):
    """Per-axis derivative bounds of F along t, u and v (the maxima over the box's corners)."""
    q = np.asarray(q, np.float64).reshape(2, 4, 3)
    d = q[1] - q[0]                    # displacement of each point, 4 x 3
    if kind == 0:
        ad = np.abs(d)
        lt = ((ad[0] + ad[1]) + ad[2]) + ad[3]
        lu = np.maximum(np.abs(q[0, 2] - q[0, 1]), np.abs(q[1, 2] - q[1, 1]))
        lv = np.maximum(np.abs(q[0, 3] - q[0, 1]), np.abs(q[1, 3] - q[1, 1]))
    else:
        ad = np.abs(d)
        lt = np.maximum(ad[0], ad[1]) + np.maximum(ad[2], ad[3])
        lu = np.maximum(np.abs(q[0, 1] - q[0, 0]), np.abs(q[1, 1] - q[1, 0]))
        lv = np.maximum(np.abs(q[0, 3] - q[0, 2]), np.abs(q[1, 3] - q[1, 2]))
    return lt.max(), lu.max(), lv.max()


def features(kind, q, delta):
    """The 16 scheduling features of one query (float32):

    0 kind (0 VF, 1 EE); 1-3 split levels m_t, m_u, m_v; 4-6 log2(1 + L/delta)
    of the derivative bounds along t, u, v; 7 signed log2(1 + |gap|/delta) of the
    root box's largest separation from the tolerance box; 8-9 the same of its
    smallest and largest side; 10 axes on which the root box meets the tolerance
    box; 11-13 the same of |F| at the parameter-space centre at t = 0, 1, 1/2;
    14 axes on which F at the centre changes sign between t = 0 and 1; 15 the
    cosine between F at the centre at t = 0 and at t = 1."""
    f = np.zeros(NF, np.float32)
    f[0] = kind
    f[1:4] = _levels(kind, q, delta)
    lt, lu, lv = _bounds(kind, q)
    f[4], f[5], f[6] = _log_ratio(lt, delta), _log_ratio(lu, delta), _log_ratio(lv, delta)
    e = _eps(kind, q)
    corners = np.array([_eval_F(kind, q, c & 1, (c >> 1) & 1, c >> 2) for c in range(8)])
    bmin, bmax = corners.min(0), corners.max(0)
    gap = np.max(np.maximum(bmin - e, -e - bmax))
    f[7] = (1.0 if gap > 0 else -1.0) * _log_ratio(gap, delta)
    w = bmax - bmin
    f[8], f[9] = _log_ratio(w.min(), delta), _log_ratio(w.max(), delta)
    f[10] = int(np.sum((bmin <= e) & (bmax >= -e)))
    c = 1.0 / 3.0 if kind == 0 else 0.5
    F0, F1, Fm = (_eval_F(kind, q, t, c, c) for t in (0.0, 1.0, 0.5))
    n0, n1, nm = (np.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) for a in (F0, F1, Fm))
    f[11], f[12], f[13] = _log_ratio(n0, delta), _log_ratio(n1, delta), _log_ratio(nm, delta)
    f[14] = int(np.sum((F0 > 0) != (F1 > 0)))
    dot = F0[0] * F1[0] + F0[1] * F1[1] + F0[2] * F1[2]
    f[15] = dot / (n0 * n1) if n0 > 0 and n1 > 0 else 0.0
    return f


def query_of(V0, V1, E, F, kind, a, b):
    """The 24 coordinates of pair (a, b): VF (vertex a, face b) or EE (edge a, edge b)."""
    if kind == 0:
        ids = [a, F[b][0], F[b][1], F[b][2]]
    else:
        ids = [E[a][0], E[a][1], E[b][0], E[b][1]]
    return np.concatenate([np.asarray(V0, np.float64)[ids].reshape(-1), np.asarray(V1, np.float64)[ids].reshape(-1)])


def pair_features(V0, V1, E, F, vf, ee, delta):
    """Features of every pair, VF pairs first (n x 16 float32)."""
    rows = [features(0, query_of(V0, V1, E, F, 0, a, b), delta) for a, b in np.asarray(vf).reshape(-1, 2)]
    rows += [features(1, query_of(V0, V1, E, F, 1, a, b), delta) for a, b in np.asarray(ee).reshape(-1, 2)]
    return np.array(rows, np.float32).reshape(-1, NF)
