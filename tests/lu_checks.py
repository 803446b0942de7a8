"""Checks shared by the GPU factorization tests: comparisons of two LU
factorizations of the same matrix computed in different summation orders
(the GPU's and the oracle's).  Plain NumPy, no GPU and no oracle calls."""
import numpy as np


def gamma(k, u):
    return k * u / (1 - k * u)


def perm_from_ipiv(ipiv):
    """Original row at each final position after the interchanges ipiv."""
    perm = np.arange(len(ipiv))
    for k, p in enumerate(ipiv):
        perm[[k, p]] = perm[[p, k]]
    return perm


def lu_difference_bound(lu_o, lu_g, pa):
    """First-order bound on |LU_g - LU_o| for two factorizations of the same
    P A_F with the same pivots.  The backward errors are measured in FP64,
    whose own evaluation error (gamma_{n+1}(u_d) (|L||U| + |P A_F|), the size
    of a binary64 factorization's backward error itself) is added; the
    factor 2 covers the second-order term."""
    n = lu_o.shape[0]
    Lo, Uo = np.tril(lu_o, -1) + np.eye(n), np.triu(lu_o)
    Lg, Ug = np.tril(lu_g, -1) + np.eye(n), np.triu(lu_g)
    LUo, LUg = np.abs(Lo) @ np.abs(Uo), np.abs(Lg) @ np.abs(Ug)
    ev = gamma(n + 1, 2.0**-53) * (LUo + LUg + 2.0 * np.abs(pa))
    E = np.abs(Lg @ Ug - pa) + np.abs(Lo @ Uo - pa) + ev
    G = np.abs(np.linalg.inv(Lo)) @ E @ np.abs(np.linalg.inv(Uo))
    return 2.0 * (np.tril(np.abs(Lo) @ np.tril(G, -1), -1) + np.triu(np.triu(G) @ np.abs(Uo)))


def active_column(af, lu_f, ipiv_f, k):
    """Column k of the active matrix just before step k chose its pivot, as
    one side computed it, rebuilt in FP64 from that side's own factors:
    s_r = a_rk - sum_{j<k} l_rj u_jk for every row r still active (indexed
    by original row), and S_r = |a_rk| + sum_{j<k} |l_rj| |u_jk|.  Rows keep
    their L entries through later interchanges (whole rows are swapped), so
    final position i >= k holds an active row."""
    n = lu_f.shape[0]
    perm = perm_from_ipiv(ipiv_f)
    Lp = lu_f[k:, :k]
    uk = lu_f[:k, k]
    a = af[perm[k:], k]
    s = a - Lp @ uk
    S = np.abs(a) + np.abs(Lp) @ np.abs(uk)
    out_s, out_S = np.zeros(n), np.zeros(n)
    out_s[perm[k:]] = s
    out_S[perm[k:]] = S
    return out_s, out_S, perm


def check_first_pivot_difference(af, lu_g, ipiv_g, lu_o, ipiv_o, k, u16, say=print):
    """At the first step k where the pivot sequences part, each side chose
    the first maximum of its own active column, and the two columns differ
    only by rounding: each side's entries are within 2 u16 S_r of the exact
    ones (16-bit L and U with unit roundoff u16: 2^-11 for binary16, 2^-8
    for bfloat16), so the two sides' within 4 u16 S_r; the two chosen rows
    are then tied up to the measured difference of the two columns (plus
    binary32 accumulation, gamma_{k+1}(u_s) S_r per entry and side)."""
    s_g, S_g, perm_g = active_column(af, lu_g, ipiv_g, k)
    s_o, S_o, perm_o = active_column(af, lu_o, ipiv_o, k)
    act = perm_o[k:]
    assert set(act.tolist()) == set(perm_g[k:].tolist())       # the same active rows
    q, p = int(perm_g[k]), int(perm_o[k])                       # GPU's and oracle's pivot rows
    S = np.maximum(S_g, S_o)
    ev = 2.0 * gamma(k + 1, 2.0**-24) * S
    # each side's choice is the maximum of its own column
    assert abs(s_g[q]) >= np.abs(s_g[act]).max() - ev[act].max()
    assert abs(s_o[p]) >= np.abs(s_o[act]).max() - ev[act].max()
    # the two columns differ by rounding only
    diff = np.abs(s_g - s_o)[act]
    assert np.all(diff <= 4.0 * u16 * S[act] + ev[act])
    # the two chosen rows are tied within that measured difference
    gap = abs(s_o[p]) - abs(s_o[q])
    slack = abs(s_o[p] - s_g[p]) + abs(s_g[q] - s_o[q]) + ev[p] + ev[q]
    say(f"  first pivot difference at step {k}: oracle's |s_p| - |s_q| = {gap:.3e} "
        f"(relative {gap / abs(s_o[p]):.2e}) <= measured column difference {slack:.3e}")
    assert gap <= slack
