"""Oracle for the paper's own algebra (test infrastructure only: nothing in the
product library imports it).  Exact integer / rational arithmetic on small rings.

The paper's scheme works in K = Q[X]/Phi_M with M = t^alpha a prime power
(Sec. 2.1), N = phi(M).  What this module computes, each from its definition:

  * Phi_M(X) = sum_{k<t} X^{k t^(alpha-1)} and reduction modulo it;
  * automorphisms sigma_d : P(X) -> P(X^d), d a unit mod M (Sec. 2.2);
  * the trace Tr(P) = sum over units d of P(X^d) (Sec. 2.3) and the partial traces
    of the tower Q = K_0 < K_1 < ... < K_alpha = K, K_i = Q(zeta_{t^i}):
    Tr_{K/K_i} sums sigma_d over d = 1 (mod t^i); on K_i, Tr_{K_i/K_j} sums the
    automorphisms d = 1 (mod t^j) taken mod t^i;
  * the dual basis (Omega*_i) of the power basis for the trace form, the coefficient
    read-out c_i = Tr(m * conj(Omega*_i)) with conj(P)(X) = P(X^(M-1)) (Sec. 4.4,
    "Partial trace extraction");
  * the two sums of the paper's lemma on partial trace extraction (Sec. 4.4), as
    plain sums of automorphisms;
  * the key switches per packed coefficient of the paper's table (Sec. 4.4, "Fast
    Packing"), from the count of Sec. 2.4 with the extraction level gamma removing
    the first gamma levels of the tower.

Polynomials are Python lists of ints or Fractions, lowest degree first; elements of
K are kept reduced (length N).
"""
from __future__ import annotations

from fractions import Fraction
from math import gcd


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    f = 2
    while f * f <= n:
        if n % f == 0:
            return False
        f += 1
    return True


def prime_factors(n: int) -> list:
    """Prime factors of n with multiplicity (the paper's omega_n)."""
    out, f = [], 2
    while f * f <= n:
        while n % f == 0:
            out.append(f)
            n //= f
        f += 1
    if n > 1:
        out.append(n)
    return out


class Ring:
    """K = Q[X]/Phi_M, M = t^alpha."""

    def __init__(self, t: int, alpha: int):
        if not is_prime(t) or alpha < 1:
            raise ValueError("M must be a prime power t^alpha, alpha >= 1")
        self.t, self.alpha = t, alpha
        self.M = t ** alpha
        self.N = self.M - self.M // t  # phi(M)
        self.units = [d for d in range(1, self.M) if gcd(d, self.M) == 1]

    # -- arithmetic ----------------------------------------------------------
    def phi(self) -> list:
        """Coefficients of Phi_M = sum_{k < t} X^(k M/t), degree N."""
        c = [0] * (self.N + 1)
        for k in range(self.t):
            c[k * (self.M // self.t)] = 1
        return c

    def reduce(self, p) -> list:
        """p mod Phi_M (Phi_M is monic of degree N: long division)."""
        p = list(p)
        phi, N = self.phi(), self.N
        for deg in range(len(p) - 1, N - 1, -1):
            c = p[deg]
            if c:
                for k, pk in enumerate(phi):
                    if pk:
                        p[deg - N + k] -= c * pk
        p = p[:N] + [0] * max(0, N - len(p))
        return p[:N]

    def mul(self, a, b) -> list:
        prod = [0] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            if x:
                for j, y in enumerate(b):
                    if y:
                        prod[i + j] += x * y
        return self.reduce(prod)

    def add(self, a, b) -> list:
        n = max(len(a), len(b))
        return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]

    def scale(self, a, c) -> list:
        return [c * x for x in a]

    def sigma(self, p, d: int) -> list:
        """P(X^d) mod Phi_M for a unit d: X^i -> X^(d i mod M) (X^M = 1 in K), then reduce."""
        if gcd(d, self.M) != 1:
            raise ValueError("d must be a unit mod M")
        out = [0] * self.M
        for i, c in enumerate(p):
            if c:
                out[(d * i) % self.M] += c
        return self.reduce(out)

    def conj(self, p) -> list:
        """conj(P)(X) = P(X^(M-1))."""
        return self.sigma(p, self.M - 1)

    # -- traces ----------------------------------------------------------------
    def trace(self, p) -> list:
        """Tr_{K/Q}(P) = sum over units d of P(X^d)."""
        acc = [0] * self.N
        for d in self.units:
            acc = self.add(acc, self.sigma(p, d))
        return acc

    def trace_down(self, p, i: int) -> list:
        """Tr_{K/K_i}(P): sum of sigma_d over the units d = 1 (mod t^i)."""
        m = self.t ** i
        acc = [0] * self.N
        for d in self.units:
            if d % m == 1 % m:
                acc = self.add(acc, self.sigma(p, d))
        return acc

    def trace_between(self, p, i: int, j: int) -> list:
        """Tr_{K_i/K_j}(P) for P in K_i, i > j: sum of sigma_d over representatives d
        of the units mod t^i with d = 1 (mod t^j) (each lifted to the unit d mod M)."""
        mi, mj = self.t ** i, self.t ** j
        reps = [d for d in range(1, mi) if gcd(d, self.t) == 1 and d % mj == 1 % mj]
        acc = [0] * self.N
        for d in reps:
            acc = self.add(acc, self.sigma(p, d))
        return acc

    def in_subfield(self, p, i: int) -> bool:
        """P in K_i <=> sigma_d(P) = P for every unit d = 1 (mod t^i)."""
        m = self.t ** i
        return all(self.sigma(p, d) == list(p) for d in self.units if d % m == 1 % m)

    # -- dual basis ------------------------------------------------------------
    def dual_basis(self) -> list:
        """conj(Omega*_i) for i < N: the elements B_i with Tr(X^j B_i) = [i = j], by
        exact Gaussian elimination on the trace-form matrix Tr(X^j X^k)."""
        N = self.N
        G = [[Fraction(self.trace(self.mul([0] * j + [1], [0] * k + [1]))[0]) for k in range(N)]
             for j in range(N)]
        # solve G b_i = e_i for every i: Gauss-Jordan on [G | I]
        A = [row[:] + [Fraction(int(r == c)) for c in range(N)] for r, row in enumerate(G)]
        for col in range(N):
            piv = next(r for r in range(col, N) if A[r][col] != 0)
            A[col], A[piv] = A[piv], A[col]
            inv = 1 / A[col][col]
            A[col] = [v * inv for v in A[col]]
            for r in range(N):
                if r != col and A[r][col] != 0:
                    f = A[r][col]
                    A[r] = [a - f * b for a, b in zip(A[r], A[col])]
        Ginv = [row[N:] for row in A]
        # B_i = sum_k (G^-1)[k][i] X^k
        return [[Ginv[k][i] for k in range(N)] for i in range(N)]


def lemma_tr_k1_k0(R: Ring, Q) -> list:
    """First sum of the lemma: sum_{k=1}^{t-1} Q(X^k)."""
    acc = [0] * R.N
    for k in range(1, R.t):
        acc = R.add(acc, R.sigma(Q, k))
    return acc


def lemma_tr_k2_k0(R: Ring, Q) -> list:
    """Second sum of the lemma: sum_{j<t} sum_{k=1}^{t-1} Q(X^(k (j t + 1)))."""
    acc = [0] * R.N
    for j in range(R.t):
        for k in range(1, R.t):
            acc = R.add(acc, R.sigma(Q, (k * (j * R.t + 1)) % R.M))
    return acc


def ramanujan_sum(M: int, t: int, i: int) -> int:
    """Sum of zeta^i over the primitive M-th roots zeta (M = t^alpha): phi(M) if
    M | i, -M/t if M/t | i but M does not, else 0 (Ramanujan's sum c_M(i))."""
    if i % M == 0:
        return M - M // t
    if i % (M // t) == 0:
        return -(M // t)
    return 0


def key_switches_per_coefficient(t: int, alpha: int, gamma: int) -> float:
    """Key switches per packed output coefficient (the paper's table in Sec. 4.4).

    Sec. 2.4 counts sum_{l in omega_{t-1}} (l - 1) key switches for Tr_{K_1/K_0} (the
    factored base level, shared by the whole packing) plus 1/t^(i-1) per coefficient
    for each higher level of the tower.  Reading (the table's values fix it): the
    levels run i = 1 .. alpha - 1, and extraction at level gamma removes Tr_{K_1/K_0}
    (gamma >= 1) and the first gamma - 1 higher levels."""
    base = sum(l - 1 for l in prime_factors(t - 1)) if gamma == 0 else 0
    start = max(1, gamma)
    return base + sum(1.0 / t ** (i - 1) for i in range(start, alpha))
