"""Solves of the semi-implicit Helmholtz-type system A x = b,
A = M + dt_m K_D (Sec. 3, eq. H_SI(1): the implicit part of H^SI; the
paper iterates every implicit equation to convergence, Sec. 8
"Runtime analysis").

Two plain solvers:
* dense: the operator is applied to every unit vector to assemble the
  matrix, then numpy.linalg.solve (tiny meshes only);
* cg   : conjugate gradients preconditioned by the diagonal mass matrix,
  iterated to a relative residual ||b - A x||_2 <= rtol ||b||_2.
The preconditioner does not change the solution, only the iterates.
"""
import numpy as np


def assemble(apply, shape):
    """Dense matrix of a linear map on arrays of the given shape."""
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = apply(e.reshape(shape)).ravel()
        e[j] = 0.0
    return A


def dense_solve(apply, b):
    A = assemble(apply, b.shape)
    return np.linalg.solve(A, b.ravel()).reshape(b.shape)


def cg(apply, b, x0, precond_diag, rtol=1e-14, maxit=10000):
    """Preconditioned CG; returns (x, iterations, final relative residual).
    precond_diag: the diagonal preconditioner's entries (z = r / diag), or a
    function r -> z (another symmetric positive definite preconditioner).

    Stops at the tolerance, or when the residual has not decreased for 50
    iterations (FP64 stagnation), keeping the best iterate."""
    pre = precond_diag if callable(precond_diag) else (lambda v: v / precond_diag)
    x = x0.copy()
    r = b - apply(x)
    bn = np.sqrt(np.sum(b * b))
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    z = pre(r)
    p = z.copy()
    rz = np.sum(r * z)
    best = (np.sqrt(np.sum(r * r)) / bn, x.copy())
    since = 0
    it = 0
    while it < maxit:
        rn = np.sqrt(np.sum(r * r)) / bn
        if rn < best[0]:
            best = (rn, x.copy())
            since = 0
        else:
            since += 1
        if rn <= rtol or since > 50:
            break
        Ap = apply(p)
        alpha = rz / np.sum(p * Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = pre(r)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    # report the true residual of the best iterate
    xb = best[1]
    rb = b - apply(xb)
    return xb, it, float(np.sqrt(np.sum(rb * rb)) / bn)
