"""The largest |eigenvalue| of a symmetric 3x3 from its characteristic cubic,
the formula the GPU's Carreau closure uses for the stress 2-norm (Eq.
strain2), restated here in numpy with the kernel's steps: the trigonometric
form with an FP32 start for c = cos(phi), two FP64 Newton steps on
4 c^3 - 3 c = r, and no answer (the kernel's Jacobi fallback) where
1 - |r| < 5e-5.  Checked against LAPACK's symmetric eigensolver on random,
traceless, D2Q9-shaped, diagonal and near-degenerate matrices."""
import numpy as np


def _cubic_norm(A):
    a00, a11, a22, a01, a02, a12 = A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]
    p1 = a01 * a01 + a02 * a02 + a12 * a12
    q = (a00 + a11 + a22) * (1.0 / 3.0)
    b00, b11, b22 = a00 - q, a11 - q, a22 - q
    p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1
    if not p2 > 0.0:
        return abs(q)
    h = p2 / 6.0
    ip = 1.0 / np.sqrt(h)
    p = h * ip
    c00, c11, c22, c01, c02, c12 = b00 * ip, b11 * ip, b22 * ip, a01 * ip, a02 * ip, a12 * ip
    r = 0.5 * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02))
    if not abs(r) < 1.0 - 5e-5:
        return None
    c = float(np.cos(np.float32(np.arccos(np.float32(r))) * np.float32(1.0 / 3.0)).astype(np.float32))
    for _ in range(2):
        c -= ((4.0 * c * c - 3.0) * c - r) / (12.0 * c * c - 3.0)
    s2 = 1.0 - c * c
    sn = np.sqrt(s2) if s2 > 0.0 else 0.0
    l1 = q + 2.0 * p * c
    l3 = q - p * (c + np.sqrt(3.0) * sn)
    l2 = 3.0 * q - l1 - l3
    return max(abs(l1), abs(l2), abs(l3))


def test_cubic_norm_matches_eigvalsh():
    rng = np.random.default_rng(5)
    worst, answered = 0.0, 0
    for i in range(20000):
        kind = i % 5
        M = rng.normal(size=(3, 3))
        A = (M + M.T) / 2.0 * 10.0 ** rng.uniform(-8, -2)
        if kind == 1:    # two eigenvalues close together
            Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            lam = rng.normal(size=3)
            lam[1] = lam[0] * (1.0 + 10.0 ** rng.uniform(-12, -1))
            A = Q @ np.diag(lam) @ Q.T * 1e-4
        elif kind == 2:  # traceless
            A = A - np.trace(A) / 3.0 * np.eye(3)
        elif kind == 3:  # the D2Q9 stress: no z row or column
            A[2, :] = 0.0
            A[:, 2] = 0.0
        elif kind == 4:  # diagonal
            A = np.diag(np.diag(A))
        v = _cubic_norm(A)
        if v is None:
            continue
        answered += 1
        exact = np.abs(np.linalg.eigvalsh(A)).max()
        worst = max(worst, abs(v - exact) / exact)
    assert answered > 15000
    assert worst < 5e-14, worst
