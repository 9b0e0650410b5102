"""Algorithmic flop model of one RGF solve (paper Sec. 3.2.3, "Computational
Complexity": O(N_B N_BS^3) per energy).

Unit: one complex b x b x b product ("GEMM-eq") = 8 b^3 real flops (four real
products of 2 b^3 each).  A complex b x b inverse (LU 8/3 b^3 + inverse
16/3 b^3) is also priced at one GEMM-eq.  Counts follow the recursions with
the products each step needs when the right-hand sides are anti-Hermitian
(the paper's symmetry X^s_ij = -conj(X^s_ji)):

  forward step 0          : 1 inverse + 2 per rhs         (x B x^dag)
  forward step i >= 1     : 2 (Schur update) + 1 inverse
                            + 4 per rhs (L x^s L^dag, x W x^dag)
                            + 1 per rhs if B has off-diagonal blocks (y_i)
  backward step i         : 6 (retarded: P, Q, R, R x, M, M x)
                            + 4 per rhs (P X^s, .P^dag, R x^s, x^s M^dag)
                            + 3 per rhs if B has off-diagonal blocks (Y_i and
                              the x B X^dag term of the upper block)
"""


def gemm_eq_rgf(n, n_rhs=2, bt_rhs=False):
    per_rhs_fwd = 4 + (1 if bt_rhs else 0)
    per_rhs_bwd = 4 + (3 if bt_rhs else 0)
    total = 1 + 2 * n_rhs
    total += (n - 1) * (3 + per_rhs_fwd * n_rhs)
    total += (n - 1) * (6 + per_rhs_bwd * n_rhs)
    return total


def rgf_flops(n, b, n_rhs=2, bt_rhs=False):
    """Real flops of one RGF solve at one energy."""
    return gemm_eq_rgf(n, n_rhs, bt_rhs) * 8 * b ** 3


def gemm_eq_w_assembly(n, n_rhs=2, want_wr=False):
    """Block products of the W-type assembly at one energy.

    Mt = I - trunc(V P^R): (V P^R)_{ij} for |i-j| <= 1 sums over k with
    |i-k| <= 1, |k-j| <= 1.  B^s = trunc(V P^s V^dag): the diagonal and upper
    blocks of (V P^s) V^dag (the lower block is minus the adjoint of the
    upper), which need (V P^s)_{ik} for k - i in {-1, 0, 1, 2}.
    W^R_ii = (X^R V)_ii: three products per block (two at the ends).
    """
    def nprod(i, j, bw_l, bw_r):
        return sum(1 for k in range(n)
                   if abs(i - k) <= bw_l and abs(k - j) <= bw_r)

    lhs = 0
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                lhs += nprod(i, j, 1, 1)
    rhs = 0
    for i in range(n):
        for k in (i - 1, i, i + 1, i + 2):          # blocks of T = V P^s
            if 0 <= k < n:
                rhs += nprod(i, k, 1, 1)
        for j in (i, i + 1):                        # blocks of T V^dag
            if j < n:
                rhs += sum(1 for k in (i - 1, i, i + 1, i + 2)
                           if 0 <= k < n and abs(k - j) <= 1)
    total = lhs + n_rhs * rhs
    if want_wr:
        total += sum(1 + (i > 0) + (i < n - 1) for i in range(n))
    return total


def w_assembly_flops(n, b, n_rhs=2, want_wr=False):
    return gemm_eq_w_assembly(n, n_rhs, want_wr) * 8 * b ** 3
