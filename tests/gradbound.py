"""Element-wise bound on a device gradient against the FP64 oracle (shared by the GPU
parity tests; its power to catch a localised error is checked on the CPU in
test_gradbound.py)."""
import numpy as np

import oracle


# Element-wise gradient bound. Element (j, k) is sum_i x_ij r_ik with r = Y - P formed
# from logits z_il = sum_j x_ij b_jl. A correct path errs in two places, each a small
# multiple of the unit roundoff u: (1) the sum over the rows, by about u sum_i |x_ij| |r_ik|;
# (2) the logits, by about u sigma_i with sigma_i = max_l (sum_j (x_ij b_jl)^2)^(1/2) (a
# sum of p rounded products), which reaches r_ik through the softmax as at most
# 2 P_ik u sigma_i. So |G - G_o| <= C_ELEM (u + u_oracle) M with
#   M_jk = sum_i |x_ij| (|r_ik| + 2 P_ik sigma_i) + |prior'(b_jk)|,
# u_oracle = 2^-53 for the FP64 oracle's own rounding. C_ELEM = 16 leaves room: a float32
# NumPy evaluation of the n=20000, p=1000, K=10 gradient stays within 0.9 u M, while one
# 16-column block off by 5e-5 relative (which the rel-L2 test alone lets through) exceeds
# 57 u M.
C_ELEM = 16.0
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def elementwise_bound(X64, y, B, prior, scale, pin, u):
    Z = X64 @ B
    P = oracle.softmax_rows(Z)
    R = oracle.onehot(y, B.shape[1]) - P
    sigma = np.sqrt((X64 ** 2) @ (B ** 2)).max(axis=1)
    M = np.abs(X64).T @ (np.abs(R) + 2.0 * P * sigma[:, None]) \
        + np.abs(oracle.log_prior_grad(B, prior, scale))
    return C_ELEM * (u + 2.0 ** -53) * M * oracle.free_mask(B.shape[0], B.shape[1], pin)


def assert_elementwise(G, G_o, X64, y, B, prior, scale, pin, u):
    bound = elementwise_bound(X64, y, B, prior, scale, pin, u)
    excess = np.abs(G - G_o) - bound
    j, k = np.unravel_index(np.argmax(excess), excess.shape)
    assert excess[j, k] <= 0.0, (f"element ({j}, {k}): |G - G_o| = {abs(G[j, k] - G_o[j, k]):.3e} "
                                 f"> bound {bound[j, k]:.3e}")
