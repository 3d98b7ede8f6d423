"""Hand-built test cases shared by the CPU pins and the GPU tests."""
import numpy as np

from oracle import hamiltonian as ham
from synth import complex_normal


def decoupled_singular_case(m=10, seed=0):
    """A, B block diagonal with a 2 x 2 leading block, so coordinates 0, 1
    (and m, m + 1) do not couple to the rest, and an orthonormal Q whose
    range is an exact +/- eigenpair of the trailing block plus the two
    S-neutral, mutually S-orthogonal vectors [e0; e1] and [e1; e0]: Q^H S Q
    has a 2 x 2 zero block.  Returns (A, B, Q, lam) with lam the exact
    positive eigenvalue in range(Q)."""
    rng = np.random.default_rng(seed)
    X = complex_normal(rng, (m, m))
    A = X @ X.conj().T / m + 2.0 * np.eye(m)
    C = complex_normal(rng, (m, m))
    B = 0.15 * (C + C.T)
    A[:2, 2:] = 0
    A[2:, :2] = 0
    B[:2, 2:] = 0
    B[2:, :2] = 0
    H = ham.assemble_h(A, B)
    idx = np.r_[2:m, m + 2:2 * m]
    w, V = np.linalg.eig(H[np.ix_(idx, idx)])
    j = int(np.argmin(np.where(w.real > 0, w.real, np.inf)))
    v = np.zeros(2 * m, complex)
    v[idx] = V[:, j]
    v /= np.linalg.norm(v)
    e = np.zeros((2 * m, 2), complex)
    e[0, 0] = e[m + 1, 0] = 1 / np.sqrt(2)
    e[1, 1] = e[m, 1] = 1 / np.sqrt(2)
    Q, _ = np.linalg.qr(np.concatenate([v[:, None], ham.apply_k_conj(v[:, None]), e], axis=1))
    return A, B, Q, float(w[j].real)
