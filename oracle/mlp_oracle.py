"""FP64 reference of the learned sampler -- TEST INFRASTRUCTURE ONLY.

Plain numpy in float64, written from the definitions of the network, the
CVAE loss and the output map; no blocking, no BF16 rounding.  Only tests,
the smoke entry and the benchmark's CPU baseline may use it.  It shares no
code with the HIP path: the parameter layout, input rows, forward pass,
back-propagation and the output map are all written out here.

Network (encoder and decoder alike): 416 inputs -> 256 ReLU -> 256 ReLU ->
16 outputs, parameters stored per network as W1 [256][416], b1, W2
[256][256], b2, W3 [16][256], b3, encoder first.  Input rows are
[v(6), 0, 0, c(396), 0 x 12] where v is the waypoint (encoder) or z
(decoder).  Loss over a batch:
    mu, lv = enc(x, c)[0:6], enc(x, c)[6:12];  z = mu + exp(lv/2) eps
    L = mean_b [ w/2 |dec(z, c)[0:6] - x|^2 + beta/2 sum(mu^2 + e^lv - 1 - lv) ]
The paper has no learned component, so nothing here is pinned by it; the
pins are finite differences, closed forms and brute force (parity of the
network itself is "parity unpinned" with respect to the paper).
"""

from __future__ import annotations

import numpy as np

IN, HID, OUT, COND, X = 416, 256, 16, 396, 6
NET = HID * IN + HID + HID * HID + HID + OUT * HID + OUT
TOTAL = 2 * NET
GRID = 2.0 ** 20


def unpack(params):
    """Flat FP64 array -> [encoder, decoder], each a dict of views."""
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (TOTAL,)
    nets = []
    for k in range(2):
        o = k * NET
        d = {}
        for name, shape in (("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
                            ("W3", (OUT, HID)), ("b3", (OUT,))):
            size = int(np.prod(shape))
            d[name] = p[o:o + size].reshape(shape)
            o += size
        nets.append(d)
    return nets


def pack(nets):
    parts = []
    for d in nets:
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            parts.append(np.asarray(d[name], dtype=np.float64).ravel())
    return np.concatenate(parts)


def rows(v, cond):
    """Input rows [v, 0, 0, cond, 0...] for per-row v [B][6] and cond [B][396]."""
    v = np.asarray(v, dtype=np.float64)
    cond = np.asarray(cond, dtype=np.float64)
    B = v.shape[0]
    Xr = np.zeros((B, IN))
    Xr[:, 0:X] = v
    Xr[:, 8:8 + COND] = cond
    return Xr


def forward(net, Xr):
    """Activations of one network: (a1, a2, out)."""
    a1 = np.maximum(Xr @ net["W1"].T + net["b1"], 0.0)
    a2 = np.maximum(a1 @ net["W2"].T + net["b2"], 0.0)
    out = a2 @ net["W3"].T + net["b3"]
    return a1, a2, out


def backward(net, Xr, a1, a2, d_out):
    """Gradients of one network from d(loss)/d(out); also d(loss)/d(input)."""
    g = {"W3": d_out.T @ a2, "b3": d_out.sum(axis=0)}
    d_a2 = d_out @ net["W3"]
    d_h2 = d_a2 * (a2 > 0)
    g["W2"] = d_h2.T @ a1
    g["b2"] = d_h2.sum(axis=0)
    d_a1 = d_h2 @ net["W2"]
    d_h1 = d_a1 * (a1 > 0)
    g["W1"] = d_h1.T @ Xr
    g["b1"] = d_h1.sum(axis=0)
    d_in = d_h1 @ net["W1"]
    return g, d_in


def cvae_loss(params, targets, cond, eps, w, beta, grads=True):
    """(loss, recon mean, kl mean, flat gradient or None) of one batch."""
    enc, dec = unpack(params)
    x = np.asarray(targets, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    B = x.shape[0]
    Xe = rows(x, cond)
    e1, e2, E = forward(enc, Xe)
    mu, lv = E[:, 0:X], E[:, X:2 * X]
    z = mu + np.exp(0.5 * lv) * eps
    Xd = rows(z, cond)
    d1, d2, D = forward(dec, Xd)
    r = D[:, 0:X] - x
    rec = 0.5 * w * np.sum(r * r, axis=1)
    kl = 0.5 * np.sum(mu * mu + np.exp(lv) - 1.0 - lv, axis=1)
    loss = float(np.mean(rec + beta * kl))
    if not grads:
        return loss, float(np.mean(rec)), float(np.mean(kl)), None
    dD = np.zeros_like(D)
    dD[:, 0:X] = w * r / B
    g_dec, d_xd = backward(dec, Xd, d1, d2, dD)
    dz = d_xd[:, 0:X]
    dE = np.zeros_like(E)
    dE[:, 0:X] = dz + beta * mu / B
    dE[:, X:2 * X] = dz * 0.5 * np.exp(0.5 * lv) * eps + beta * 0.5 * (np.exp(lv) - 1.0) / B
    g_enc, _ = backward(enc, Xe, e1, e2, dE)
    return loss, float(np.mean(rec)), float(np.mean(kl)), pack([g_enc, g_dec])


def decode(params, cond, eps):
    """Raw decoder outputs [count][6] for one condition and prior draws z = eps."""
    _, dec = unpack(params)
    eps = np.asarray(eps, dtype=np.float64)
    c = np.broadcast_to(np.asarray(cond, dtype=np.float64), (eps.shape[0], COND))
    return forward(dec, rows(eps, c))[2][:, 0:X]


def adam(params, grads, m, v, step, lr, b1, b2, eps):
    """One Adam step (bias-corrected moments); returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grads
    v = b2 * v + (1.0 - b2) * grads * grads
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def finish(raw, boxes, fallback):
    """Raw outputs [count][6] -> SoA states [6][count] and the rejected count.

    Position sigmoid(u); velocity w / sqrt(1 + |w|^2); both rounded to the
    nearest multiple of 2^-20 (ties to even).  Rejected (replaced by the
    fallback column): a non-finite value, a rounded velocity with
    |q|^2 > 2^40, or a rounded position inside a closed box."""
    raw = np.asarray(raw, dtype=np.float64)
    fallback = np.asarray(fallback, dtype=np.float32)
    boxes = np.asarray(boxes, dtype=np.float64).reshape(-1, 6)
    bq = np.rint(boxes * GRID).astype(np.int64)
    count = raw.shape[0]
    out = np.zeros((6, count), dtype=np.float32)
    rejected = 0
    for b in range(count):
        u = raw[b, 0:6]
        bad = not np.all(np.isfinite(u))
        q = np.zeros(6, dtype=np.int64)
        if not bad:
            with np.errstate(over="ignore"):
                pos = 1.0 / (1.0 + np.exp(-u[0:3]))
            vel = u[3:6] / np.sqrt(1.0 + float(u[3] * u[3] + u[4] * u[4] + u[5] * u[5]))
            q[0:3] = np.rint(pos * GRID).astype(np.int64)
            q[3:6] = np.rint(vel * GRID).astype(np.int64)
            if int(q[3] * q[3] + q[4] * q[4] + q[5] * q[5]) > (1 << 40):
                bad = True
            for k in range(bq.shape[0]):
                if all(bq[k, a] <= q[a] <= bq[k, 3 + a] for a in range(3)):
                    bad = True
                    break
        if bad:
            rejected += 1
            out[:, b] = fallback[:, b]
        else:
            out[:, b] = (q.astype(np.float64) / GRID).astype(np.float32)
    return out, rejected
