"""Test infrastructure: the reference of one Adam step on every program's
constants, in binary64 (Kingma & Ba, "Adam: A Method for Stochastic
Optimization", 2015, Alg. 1), with the best point kept per program.

Constant optimisation is what the paper names as the next thing to integrate
with GPU evaluation (Section 5); it is driven by the fitness gradient.  Per
program i (row of every array):
  * if fitness[i] < best_f[i]: best_c[i] = consts[i], best_f[i] = fitness[i]
    (the fitness belongs to the constants the gradient was taken at);
  * if fitness[i] is not finite: consts[i] = best_c[i], moments reset to 0;
  * otherwise, per constant with a finite gradient g (and g^2 within the
    binary32 range, the device's moment type):
        m = b1 m + (1 - b1) g,   v = b2 v + (1 - b2) g^2,
        c = c - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Only tests and the benchmark's CPU leg use this module.
"""
import numpy as np


def adam_step(consts, grad, fitness, m1, m2, best_c, best_f, t, lr, beta1=0.9, beta2=0.999,
              eps=1e-12):
    """Return new (consts, m1, m2, best_c, best_f); inputs are not modified."""
    c = np.array(consts, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    f = np.asarray(fitness, dtype=np.float64)
    m1 = np.array(m1, dtype=np.float64)
    m2 = np.array(m2, dtype=np.float64)
    bc = np.array(best_c, dtype=np.float64)
    bf = np.array(best_f, dtype=np.float64)
    for i in range(c.shape[0]):
        if f[i] < bf[i]:
            bc[i] = c[i]
            bf[i] = f[i]
        if not np.isfinite(f[i]):
            c[i] = bc[i]
            m1[i] = 0.0
            m2[i] = 0.0
            continue
        for j in range(c.shape[1]):
            g32 = np.float32(g[i, j])
            with np.errstate(over="ignore", invalid="ignore"):
                if not np.isfinite(g32 * g32):
                    continue
            m1[i, j] = beta1 * m1[i, j] + (1.0 - beta1) * g[i, j]
            m2[i, j] = beta2 * m2[i, j] + (1.0 - beta2) * g[i, j] ** 2
            mhat = m1[i, j] / (1.0 - beta1 ** t)
            vhat = m2[i, j] / (1.0 - beta2 ** t)
            c[i, j] -= lr * mhat / (np.sqrt(vhat) + eps)
    return c, m1, m2, bc, bf
