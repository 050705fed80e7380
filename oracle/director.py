"""Oracle-side director and defect extraction, written plainly with numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What it encodes (sec. II, Eq. Qtensor and the text after it; sec. IV, the
GUI's director and defect display):
  * the director is the eigenvector of Q for its largest eigenvalue (which
    equals S for the uniaxial and biaxial forms of Eq. Qtensor);
  * a defect site is a simulated site whose largest eigenvalue lies below a
    threshold.
Reading: n and -n are the same director; the returned sign makes the
component of largest magnitude positive (the first of equal magnitudes).
Sites inside objects, and sites with Q = 0 (no preferred axis), get n = 0
and largest eigenvalue 0; a site inside an object is never a defect.
"""
from __future__ import annotations

import numpy as np


def full_Q(q):
    """(N, 3, 3) tensors from q of shape (5, N), Qzz = -Qxx - Qyy."""
    q = np.asarray(q, dtype=np.float64).reshape(5, -1)
    Q = np.empty((q.shape[1], 3, 3))
    Q[:, 0, 0], Q[:, 0, 1], Q[:, 0, 2] = q[0], q[1], q[2]
    Q[:, 1, 0], Q[:, 1, 1], Q[:, 1, 2] = q[1], q[3], q[4]
    Q[:, 2, 0], Q[:, 2, 1], Q[:, 2, 2] = q[2], q[4], -q[0] - q[3]
    return Q


def canonical_sign(n):
    """Flips each column of n (3, N) so its largest-magnitude component is positive."""
    n = np.array(n, dtype=np.float64)
    idx = np.argmax(np.abs(n), axis=0)
    sgn = np.sign(n[idx, np.arange(n.shape[1])])
    sgn[sgn == 0] = 1.0
    return n * sgn


def directors(q, types, threshold):
    """Returns (n (3, N), lambda_max (N,), eigenvalues (N, 3) ascending,
    defect (N,) bool) of the field q (5, N)."""
    types = np.asarray(types).reshape(-1)
    Q = full_Q(q)
    w, V = np.linalg.eigh(Q)            # ascending eigenvalues, eigenvectors in columns
    lam = w[:, 2].copy()
    n = canonical_sign(V[:, :, 2].T)
    inside = types == 2
    zero = np.all(Q.reshape(-1, 9) == 0.0, axis=1)
    n[:, inside | zero] = 0.0
    lam[inside | zero] = 0.0
    w[inside] = 0.0
    defect = (~inside) & (lam < threshold)
    return n, lam, w, defect
