"""Plain FP64 reference of the membrane surrogate: per-vertex 1-ring
features, a small multilayer perceptron, its gradient and Adam.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg,
never by the library.  It shares no code with the HIP path.

The paper has no learned component; this follows the surrogate the workload
description asks for (a learned replacement of the membrane bending force,
Eq. (19), and local-area force, Eq. (17)), with these readings:

  - ring: the neighbours of vertex v in counter-clockwise order seen from
    outside (the order the outward-oriented triangles give), starting at the
    neighbour with the smallest mesh index, so the order is fixed by the
    topology alone;
  - local frame: n = normalised sum of u_k x u_{k+1} over the ring (u_k the
    nearest-image vector from v to its k-th neighbour), e1 = the component
    of u_0 normal to n, normalised, e2 = n x e1; R has rows (e1, e2, n);
  - inputs (20): R u_k / ell for the first six ring slots (a degree-5 vertex
    leaves slot 6 zero), then c_dev (A - A0)/A0 and c_dev (V - V0)/V0 of the
    vertex's cell; vertices of degree other than 5 or 6 always use the plain
    forces;
  - network: 20 -> 128 -> 128 -> 128 -> 3, SiLU after each hidden layer,
    parameters stored as [W1 (128x20, row = output), b1, W2, b2, W3, b3, W4
    (3x128), b4] = 36,099 floats;
  - precision: weights, inputs and every hidden activation are rounded to
    bfloat16 (round to nearest even) where they enter a product, products
    are accumulated exactly here (FP64) and in FP32 on the GPU, biases and
    SiLU are applied in full precision;
  - output: force = s_F R^T y (y in the local frame);
  - loss: mean over the batch and the 3 components of (y - t)^2, t the
    target force in the local frame divided by s_F;
  - optimiser: Adam (Kingma & Ba, 2015) with bias correction.
"""
import numpy as np

N_IN, N_HID, N_OUT = 20, 128, 3
SHAPES = [(N_HID, N_IN), (N_HID, N_HID), (N_HID, N_HID), (N_OUT, N_HID)]
N_PARAMS = sum(o * i + o for o, i in SHAPES)  # 36,099


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    """List of (W [out][in], b [out]) views of the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for no, ni in SHAPES:
        W = p[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = p[o:o + no]
        o += no
        out.append((W, b))
    assert o == N_PARAMS
    return out


def init_params(rng):
    """He-style initial weights (normal, std sqrt(2/fan_in)), zero biases."""
    parts = []
    for no, ni in SHAPES:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / ni), no * ni))
        parts.append(np.zeros(no))
    return np.concatenate(parts).astype(np.float32)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def silu_grad(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, rounding=True):
    """Y [n][3] and the pre-activations / activations of every layer."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params)
    H = [np.asarray(X, dtype=np.float64)]
    Z = []
    for li, (W, b) in enumerate(layers):
        z = r(H[-1]) @ r(W).T + b
        Z.append(z)
        H.append(silu(z) if li < len(layers) - 1 else z)
    return H[-1], dict(H=H, Z=Z)


def loss_and_grad(params, X, T, rounding=True):
    """Mean squared error over the batch and outputs, and its gradient with
    respect to the flat parameters (same rounding points as the forward
    pass: every operand entering a product is rounded to bfloat16)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params)
    Y, c = forward(params, X, rounding)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    loss = float(np.mean((Y - T) ** 2))
    dz = 2.0 * (Y - T) / (n * N_OUT)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dW = r(dz).T @ r(c["H"][li])
        db = dz.sum(axis=0)
        grads[li] = (dW, db)
        if li > 0:
            dh = r(dz) @ r(W)
            dz = dh * silu_grad(c["Z"][li - 1])
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ features
def rings(tri, nv):
    """Counter-clockwise neighbour rings (outward view) starting at the
    smallest neighbour index; None for a vertex whose ring is not a cycle."""
    nxt = [dict() for _ in range(nv)]
    for a, b, c in np.asarray(tri):
        for v, p, q in ((a, b, c), (b, c, a), (c, a, b)):
            nxt[v][int(p)] = int(q)
    out = []
    for v in range(nv):
        d = nxt[v]
        start = min(d)
        ring, k = [start], d[start]
        while k != start and len(ring) <= len(d):
            ring.append(k)
            k = d[k]
        out.append(ring if (k == start and len(ring) == len(d)) else None)
    return out


def frame(u):
    """Rows (e1, e2, n) of the local frame of a ring of vectors u [d][3]."""
    d = u.shape[0]
    nrm = sum(np.cross(u[k], u[(k + 1) % d]) for k in range(d))
    n = nrm / np.linalg.norm(nrm)
    t = u[0] - np.dot(u[0], n) * n
    e1 = t / np.linalg.norm(t)
    e2 = np.cross(n, e1)
    return np.array([e1, e2, n])


def features(pos, box, ring, A, A0, V, V0, ell, c_dev):
    """Inputs X [nv][20], frames R [nv][3][3] and the surrogate mask (degree
    5 or 6) of one cell whose vertices are pos [nv][3] (wrapped, box L)."""
    pos = np.asarray(pos, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)
    nv = pos.shape[0]
    X = np.zeros((nv, N_IN))
    R = np.zeros((nv, 3, 3))
    ok = np.zeros(nv, dtype=bool)
    for v in range(nv):
        rg = ring[v]
        u = pos[rg] - pos[v]
        u -= L * np.round(u / L)
        R[v] = frame(u)
        if len(rg) in (5, 6):
            ok[v] = True
            loc = (R[v] @ u.T).T / ell
            X[v, :3 * len(rg)] = loc.ravel()
        X[v, 18] = c_dev * (A - A0) / A0
        X[v, 19] = c_dev * (V - V0) / V0
    return X, R, ok


def surrogate_forces(params, X, R, s_F, rounding=True):
    """Forces s_F R^T y of the network in the global frame, [nv][3]."""
    Y, _ = forward(params, X, rounding)
    return s_F * np.einsum("nij,ni->nj", R, Y)
