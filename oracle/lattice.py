"""Lattice algebra of the D3Q27 cuboid lattice (oracle; test infrastructure only).

Everything here is an explicit matrix built from its definition in the paper:

* velocity set               -- eq. 1a-c (Sec. 2.1)
* raw-moment ordering m      -- the list of countable raw moments after eq. 56
* cubic moment basis P       -- eq. for P in Sec. 3.1, entries ebar_x^m ebar_y^n ebar_z^p
* scaling S = diag(r^n s^p)  -- eq. 58-59; S^-1 of eq. 61
* cuboid moment basis Q      -- eq. 57 (entries e_x^m e_y^n e_z^p); Q = S P
* non-orthogonal basis T     -- eq. 4-5; T = B Q
* B (moment combinations)    -- eq. 5 / the combinations of App. D; B^-1 as the
                                 segregation formulas of App. D
* frame transformation F(u)  -- binomial expansion of the central moments of
                                 eq. 3a in terms of raw moments (App. C);
                                 F^-1 = F(-u) (remark at the end of Sec. 3.1)
"""

import functools
import math

import torch

DT = torch.float64

# eq. 1a-c: integer direction components (ebar); e = (ebar_x, r*ebar_y, s*ebar_z).
EX = (0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1)
EY = (0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1)
EZ = (0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1)
Q27 = 27

# Raw/central moment ordering (m, n, p) of the vector m listed after eq. 56 and
# of m^c in Sec. 3.1: k000, k100, k010, k001, k110, k101, k011, k200, k020, k002,
# k120, k102, k210, k012, k201, k021, k111, k220, k202, k022, k211, k121, k112,
# k122, k212, k221, k222.
MOMENTS = (
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2),
    (2, 0, 1), (0, 2, 1), (1, 1, 1), (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 1, 1),
    (1, 2, 1), (1, 1, 2), (1, 2, 2), (2, 1, 2), (2, 2, 1), (2, 2, 2),
)
MIDX = {mnp: i for i, mnp in enumerate(MOMENTS)}


@functools.lru_cache(maxsize=None)
def ebar():
    """Integer direction vectors, shape (27, 3) (eq. 1 with r = s = 1)."""
    return torch.tensor(list(zip(EX, EY, EZ)), dtype=torch.int64)


@functools.lru_cache(maxsize=None)
def velocities(r, s):
    """Cuboid particle velocities e_alpha = (ebar_x, r ebar_y, s ebar_z), eq. 1a-c."""
    e = ebar().to(DT)
    return e * torch.tensor([1.0, r, s], dtype=DT)


@functools.lru_cache(maxsize=None)
def opposite():
    """Index abar of the direction with e_abar = -e_a (used by bounce-back, Sec. 4)."""
    eb = ebar()
    out = []  # returned as a tuple (cached)
    for a in range(Q27):
        matches = [b for b in range(Q27) if bool(torch.all(eb[b] == -eb[a]))]
        assert len(matches) == 1
        out.append(matches[0])
    return tuple(out)


def moment_matrix(e):
    """Rows e_x^m e_y^n e_z^p over the directions, in the MOMENTS ordering."""
    rows = []
    for (m, n, p) in MOMENTS:
        rows.append(e[:, 0] ** m * e[:, 1] ** n * e[:, 2] ** p)
    return torch.stack(rows)


@functools.lru_cache(maxsize=None)
def P_matrix():
    """Cubic-lattice raw-moment basis P (Sec. 3.1): m = P f on the cubic lattice."""
    return moment_matrix(ebar().to(DT))


@functools.lru_cache(maxsize=None)
def S_diag(r, s):
    """Diagonal of the scaling matrix S: entry r^n s^p for moment k'_mnp (eq. 59)."""
    return torch.tensor([float(r) ** n * float(s) ** p for (_, n, p) in MOMENTS], dtype=DT)


@functools.lru_cache(maxsize=None)
def Q_matrix(r, s):
    """Cuboid raw-moment basis Q of eq. 57 (entries e_x^m e_y^n e_z^p)."""
    return moment_matrix(velocities(r, s))


@functools.lru_cache(maxsize=None)
def P_inverse():
    """P^-1 by dense inversion (App. G prints it term by term)."""
    return torch.linalg.inv(P_matrix())


# Combinations of eq. 5 / eq. 7 in the n ordering: each entry lists
# (coefficient, moment) pairs.  Index 7, 8, 9 are the two deviatoric diagonal
# combinations and the trace (k_2d1, k_2d2, k_2s of App. D).
N_COMBINATIONS = (
    ((1, (0, 0, 0)),),
    ((1, (1, 0, 0)),),
    ((1, (0, 1, 0)),),
    ((1, (0, 0, 1)),),
    ((1, (1, 1, 0)),),
    ((1, (1, 0, 1)),),
    ((1, (0, 1, 1)),),
    ((1, (2, 0, 0)), (-1, (0, 2, 0))),                     # 7: 2d1
    ((1, (2, 0, 0)), (-1, (0, 0, 2))),                     # 8: 2d2
    ((1, (2, 0, 0)), (1, (0, 2, 0)), (1, (0, 0, 2))),      # 9: 2s
    ((1, (1, 2, 0)), (1, (1, 0, 2))),                      # 10: 3s1
    ((1, (2, 1, 0)), (1, (0, 1, 2))),                      # 11: 3s2
    ((1, (2, 0, 1)), (1, (0, 2, 1))),                      # 12: 3s3
    ((1, (1, 2, 0)), (-1, (1, 0, 2))),                     # 13: 3m1
    ((1, (2, 1, 0)), (-1, (0, 1, 2))),                     # 14: 3m2
    ((1, (2, 0, 1)), (-1, (0, 2, 1))),                     # 15: 3m3
    ((1, (1, 1, 1)),),
    ((1, (2, 2, 0)), (1, (2, 0, 2)), (1, (0, 2, 2))),      # 17: 4s
    ((1, (2, 2, 0)), (1, (2, 0, 2)), (-1, (0, 2, 2))),     # 18: 4d1
    ((1, (2, 2, 0)), (-1, (2, 0, 2))),                     # 19: 4d2
    ((1, (2, 1, 1)),),
    ((1, (1, 2, 1)),),
    ((1, (1, 1, 2)),),
    ((1, (1, 2, 2)),),
    ((1, (2, 1, 2)),),
    ((1, (2, 2, 1)),),
    ((1, (2, 2, 2)),),
)
N_2D1, N_2D2, N_2S = 7, 8, 9


@functools.lru_cache(maxsize=None)
def B_matrix():
    """B of T = B Q: combines moments (MOMENTS ordering) into the n ordering of eq. 7."""
    B = torch.zeros(Q27, Q27, dtype=DT)
    for row, terms in enumerate(N_COMBINATIONS):
        for c, mnp in terms:
            B[row, MIDX[mnp]] = c
    return B


@functools.lru_cache(maxsize=None)
def B_inverse():
    """B^-1: the segregation formulas that close App. D, as a matrix (by inversion)."""
    return torch.linalg.inv(B_matrix())


@functools.lru_cache(maxsize=None)
def T_matrix(r, s):
    """Non-orthogonal basis T of eq. 4-5, built directly from its monomials."""
    e = velocities(r, s)
    ex, ey, ez = e[:, 0], e[:, 1], e[:, 2]
    one = torch.ones(Q27, dtype=DT)
    x2, y2, z2 = ex * ex, ey * ey, ez * ez
    rows = [
        one, ex, ey, ez, ex * ey, ex * ez, ey * ez,
        x2 - y2, x2 - z2, x2 + y2 + z2,
        ex * y2 + ex * z2, x2 * ey + ey * z2, x2 * ez + y2 * ez,
        ex * y2 - ex * z2, x2 * ey - ey * z2, x2 * ez - y2 * ez,
        ex * ey * ez,
        x2 * y2 + x2 * z2 + y2 * z2, x2 * y2 + x2 * z2 - y2 * z2, x2 * y2 - x2 * z2,
        x2 * ey * ez, ex * y2 * ez, ex * ey * z2,
        ex * y2 * z2, x2 * ey * z2, x2 * y2 * ez, x2 * y2 * z2,
    ]
    return torch.stack(rows)


def _binomial_axis(u):
    """Per-axis 3x3 shift matrices A[i, j] = C(i, j) (-u)^(i-j) for j <= i, shape (N, 3, 3)."""
    n = u.shape[0]
    A = torch.zeros(n, 3, 3, dtype=u.dtype)
    for i in range(3):
        for j in range(i + 1):
            A[:, i, j] = math.comb(i, j) * (-u) ** (i - j)
    return A


@functools.lru_cache(maxsize=None)
def _tensor_to_moment_index():
    """Position of each MOMENTS entry in the flattened (i, j, k) tensor order (i*9 + j*3 + k)."""
    return torch.tensor([m * 9 + n * 3 + p for (m, n, p) in MOMENTS])


def frame_matrix(u):
    """Frame transformation F(u): m^c = F(u) m, one 27x27 matrix per node.

    From eq. 3a, (e - u)^m expanded by the binomial theorem gives
    k_mnp = sum_{i<=m, j<=n, k<=p} C(m,i) C(n,j) C(p,k) (-u_x)^(m-i) (-u_y)^(n-j)
    (-u_z)^(p-k) k'_ijk; App. C lists the same expansion term by term.  The
    27x27 matrix is the product of the three per-axis 3x3 shift matrices,
    re-indexed into the MOMENTS ordering.  ``u`` has shape (N, 3); the result
    has shape (N, 27, 27).
    """
    ax = _binomial_axis(u[:, 0])
    ay = _binomial_axis(u[:, 1])
    az = _binomial_axis(u[:, 2])
    full = torch.einsum("nab,ncd,nef->nacebdf", ax, ay, az).reshape(u.shape[0], 27, 27)
    idx = _tensor_to_moment_index()
    return full[:, idx][:, :, idx]


def frame_matrix_inverse(u):
    """F^-1(u) = F(-u) (stated at the end of Sec. 3.1 and used in App. E)."""
    return frame_matrix(-u)
