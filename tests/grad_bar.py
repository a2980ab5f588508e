"""Per-element tolerance of the backward kernel (crbm_grad) against the
oracle's FP64 gradient.

For a parameter p the kernel returns sum_b g_b dF(x_b)/dtheta_p, where every
per-sample derivative of W and h_bias is -sum sigma(a) v over hidden units
(each term <= 0) and that of v_bias is -sum v (exact).  The pre-activations
and sigma are FP64; sigma is kept in LDS as FP64, or rounded once to float32
when K L^2 doubles do not fit.  A relative error r of every sigma therefore
moves the result by at most r A_p with

    A_p = sum_b |g_b dF(x_b)/dtheta_p|,

the oracle's vector-Jacobian product with |g|.  The final rounding to float32
adds 2^-24 |ref|.  The bar per element is

    |got - ref| <= 1e-5 |ref| + (r_sigma + r_g) A_p,

r_sigma = 2^-24 (float32 sigma) or 2^-45 (FP64 sigma: pre-activation sums of
at most C Lw^2 + 1 terms, exp and division, far below 2^-45 relative), and r_g
the relative error of the cotangents g handed to the kernel (0 when the test
passes the oracle the same float32 values, 2^-24 when torch rounds a float64
cotangent to float32 in the autograd backward).
"""
import numpy as np

R_SIG32 = 2.0 ** -24
R_SIG64 = 2.0 ** -45


def sigma_is_fp64(K, C, Lw, L, banks=1):
    """Mirror of the kernel's choice: sigma in FP64 when it fits 160 KiB of LDS."""
    return K * L * L * 8 + banks * K * C * Lw * Lw * 4 + C * L * L + 16 <= 160 * 1024


def grad_abs(orc, m, x, g):
    """A_p for every parameter: the oracle's gradient with |g|."""
    return orc.grad(m, x, np.abs(np.asarray(g, np.float64)))


def assert_grad_close(got, ref, A, r):
    got = np.asarray(got, np.float64).reshape(ref.shape)
    tol = 1e-5 * np.abs(ref) + r * np.abs(A)
    err = np.abs(got - ref)
    bad = err > tol
    assert not bad.any(), (
        f"{int(bad.sum())} of {bad.size} elements outside the bar; worst err {err.max():.3e}, "
        f"worst err/tol {(err / np.maximum(tol, 1e-300)).max():.3f}")
