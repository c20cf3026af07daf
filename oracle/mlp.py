"""CPU oracle of the learned work-item cost model -- TEST INFRASTRUCTURE ONLY.

Only the test suite and the CPU-baseline leg of the benchmark may import this
module; the library never does and shares no code with it.

The cost model is not part of the paper, which leaves better load balancing
of its parallel pair counting to future work (Sect. 4.2, 4.3 and 6).  What is
computed here is the textbook definition, in float64:

* a multilayer perceptron 4 -> 64 -> 64 -> 64 -> 1 with ReLU after each hidden
  layer and a linear output:  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
  h3 = relu(W3 h2 + b3), y = W4 . h3 + b4;
* inputs standardised as (x - mean) / std per feature, the output scaled back
  as y * std_t + mean_t;
* the loss 0.5 * sum over samples of (y - t)^2 in standardised units and its
  gradient by the chain rule (back-propagation), ReLU derivative 1 where the
  activation is positive, else 0;
* the Adam update (Kingma & Ba, 2015): m = b1 m + (1 - b1) g,
  v = b2 v + (1 - b2) g^2, p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
  with g the gradient averaged over the minibatch.

Parameters use the packed layout of the library interface:
W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4.
"""
import numpy as np

NF, NH = 4, 64
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH,)), ("b4", ())]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params):
    """Split the packed vector into named float64 arrays (copies)."""
    p = np.asarray(params, dtype=np.float64).ravel()
    if p.size != NPARAM:
        raise ValueError(f"expected {NPARAM} parameters, got {p.size}")
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape).copy()
        o += n
    return out


def pack(named):
    return np.concatenate([np.asarray(named[name], dtype=np.float64).ravel() for name, _ in SIZES])


def standardise(feat, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(feat, dtype=np.float64) - norm[0:4]) / norm[4:8]


def forward(params, xs):
    """Network output for standardised inputs xs (m, 4); returns y (m,) and the activations."""
    P = unpack(params)
    xs = np.asarray(xs, dtype=np.float64)
    h1 = np.maximum(xs @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    h3 = np.maximum(h2 @ P["W3"].T + P["b3"], 0.0)
    y = h3 @ P["W4"] + P["b4"]
    return y, (xs, h1, h2, h3)


def predict(params, norm, feat):
    """Prediction in target units: std_t * net((feat - mean) / std) + mean_t."""
    norm = np.asarray(norm, dtype=np.float64)
    y, _ = forward(params, standardise(feat, norm))
    return y * norm[9] + norm[8]


def loss_and_grad(params, norm, feat, target):
    """0.5 * sum (y - t)^2 in standardised units and its gradient (packed layout)."""
    norm = np.asarray(norm, dtype=np.float64)
    P = unpack(params)
    y, (x, h1, h2, h3) = forward(params, standardise(feat, norm))
    t = (np.asarray(target, dtype=np.float64) - norm[8]) / norm[9]
    d = y - t
    loss = 0.5 * float(np.sum(d * d))
    g = {"W4": h3.T @ d, "b4": np.sum(d)}
    dz3 = np.outer(d, P["W4"]) * (h3 > 0)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ P["W3"]) * (h2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (h1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(params, grad, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m1, m2)."""
    g = np.asarray(grad, dtype=np.float64)
    m1 = b1 * np.asarray(m1, dtype=np.float64) + (1.0 - b1) * g
    m2 = b2 * np.asarray(m2, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m1 / (1.0 - b1 ** step)
    vhat = m2 / (1.0 - b2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m1, m2


def fit_norm(feat, target, floor=1e-3):
    """Per-feature and target mean / population standard deviation (floored)."""
    f = np.asarray(feat, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    return np.concatenate([f.mean(axis=0), np.maximum(f.std(axis=0), floor),
                           [t.mean(), max(t.std(), floor)]])
