"""Oracle for the paper's own server pipeline on ciphertexts (TEST INFRASTRUCTURE ONLY:
only the test suite, the smoke check and the CPU-baseline leg of the benchmark may use
it; the HIP library never imports or calls it).

Scheme (paper Sec. 2.1-2.4, 4.2, 4.4): RLWE over the discrete torus with q = 2^64,
ring Z_q[X]/Phi_M, M = t^alpha, N = phi(M).  A ciphertext (a, b) of the message mu
satisfies b - s a = mu + e; a message m in Z_p is the torus value m 2^64 / p and is
decoded by rounding p (b - s a) / 2^64.  Arithmetic is exact modulo 2^64 (numpy uint64
wraps), polynomials are uint64 arrays of the N power-basis coefficients.

What is computed, each from its definition:
  * the ring product: the full integer convolution, folded modulo X^M - 1 and then
    modulo Phi_M = sum_{k<t} X^(k M/t), i.e. X^(N + r) = -sum_{k<t-1} X^(k M/t + r)
    for r < M/t;
  * automorphisms sigma_d: X^i -> X^(d i mod M) (Sec. 2.2);
  * key switching with a gadget of base D and depth l (Sec. 4.2; D = 2^log_d, or any
    even base such as the paper's 310): the key for sigma_d is the l encryptions of
    s(X^d) g_i with g_i = round(2^64 / D^i) (exactly 2^64 / D^i for a power of two); a
    ciphertext under s(X^d) is decomposed into l balanced digit polynomials of its
    mask (the mask as a torus value rounded to a multiple of 1 / D^l, written in
    balanced base D) and recombined with the key;
  * partial trace extraction (Sec. 4.4, the lemma on partial trace extraction): the
    client sends encryptions of m(X^d) for d in the level-gamma set ({1..t-1} for
    gamma = 1, {k (j t + 1)} for gamma = 2); the server forms, for every coefficient
    i, E_i = u sum_d ct(m(X^d)) (M conj(Omega*_i))(X^d) with u = M^-1 mod p, where
    M conj(Omega*_i) = X^(M-i) - X^(M/t - r), r = i mod M/t (two terms modulo
    X^M - 1: the dual basis of the power basis for the trace form, pinned against
    exact Gaussian elimination in oracle/native.py);
  * the integer-weight linear layer on the extracted rows, F_o = sum_i W[o][i] E_i
    (Sec. 4.4 "Convolution": the convolution is a matrix product over rows whose
    entries are ciphertext coefficients), with the shuffle folded into W's rows;
  * fast packing (Sec. 2.4, 4.4): phi(t^beta) rows F_o, each with
    Tr_{K/K_gamma}(dec F_o) = y_o 2^64/p, are packed into one ciphertext of
    sum_o y_o X^(o M / t^beta).  This oracle's packing (a reading: the paper names
    the technique but not its steps) builds the result up the tower:
      leaves  l_e = sum_{j < phi(t^gamma)} X^(j M/t^gamma) F_(e + j T), T = t^(beta-gamma);
      merge   at level i (gamma <= i < beta) t sub-packs y_k valid at level i
              (Tr_{K/K_i}(dec y_k) = Y_k) become Y = sum_m tau_i^m(v_m) with
              v_m = sum_k X^(k (M/t^(i+1) - m M/t)) y_k and tau_i = sigma_(1 + t^i),
              evaluated as S = v_(t-1), S = v_m + tau_i(S) (t - 1 key switches); then
              Tr_{K/K_(i+1)}(dec Y) = sum_k theta^k Y_k, theta = X^(M/t^(i+1));
      trace   Tr_{K/K_beta} as prod over levels j = beta..alpha-1 of
              sum_{k<t} tau_j^k, each S = P, S = P + tau_j(S) (t - 1 key switches),
              the levels taken from j = alpha-1 down (the factors commute; the
              order fixes which ciphertext, among equally valid ones, comes out).
    Key switches per packed ciphertext: t^(beta-gamma) - 1 + (alpha - beta)(t - 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U64 = np.uint64


@dataclass
class NativeParams:
    t: int
    alpha: int
    gamma: int        # partial trace extraction level (1 or 2)
    beta: int         # packing level: phi(t^beta) coefficients per packed ciphertext
    log_d: int        # gadget base D = 2^log_d (when base is 0)
    l: int            # gadget depth
    log_p: int        # message modulus p = 2^log_p
    sigma: float      # error standard deviation in units of 2^-64 (the paper's Delta 2^64)
    base: int = 0     # an even gadget base that is not a power of two (0: D = 2^log_d)
    M: int = field(init=False)
    N: int = field(init=False)

    def __post_init__(self):
        assert self.t >= 3 and all(self.t % f for f in range(2, int(self.t ** 0.5) + 1)), "t: odd prime"
        assert 1 <= self.gamma <= 2 and self.gamma <= self.beta <= self.alpha - 1
        assert self.log_p < 32
        if self.base:
            assert self.base % 2 == 0 and 4 <= self.base <= 1 << 16 and self.base ** self.l < 1 << 63
        else:
            assert self.log_d * self.l < 64
        self.M = self.t ** self.alpha
        self.N = self.M - self.M // self.t

    @property
    def D(self) -> int:
        return self.base or 1 << self.log_d

    def gadget(self, i: int) -> int:
        """g_i = round(2^64 / D^i), i = 1..l."""
        return ((1 << 65) // self.D ** i + 1) // 2

    @property
    def Mt(self) -> int:
        return self.M // self.t

    @property
    def p(self) -> int:
        return 1 << self.log_p

    @property
    def n_pack(self) -> int:
        """Coefficients per packed ciphertext: phi(t^beta)."""
        return (self.t - 1) * self.t ** (self.beta - 1)

    def powers(self) -> list:
        """The exponents d of the client's encrypted powers m(X^d) at level gamma."""
        t = self.t
        if self.gamma == 1:
            return list(range(1, t))
        return [(k * (j * t + 1)) % self.M for k in range(1, t) for j in range(t)]

    def u(self) -> int:
        """M^-1 mod p, balanced (|u| <= p/2: the same message, the smallest noise
        growth), as an integer modulo 2^64."""
        u = pow(self.M, -1, self.p)
        return (u - self.p if u > self.p // 2 else u) % 2 ** 64

    def taus(self) -> list:
        """Galois elements of the key-switching keys: 1 + t^i for i = gamma .. alpha-1."""
        return [(1 + self.t ** i) % self.M for i in range(self.gamma, self.alpha)]

    def key_switches_per_pack(self) -> int:
        return self.t ** (self.beta - self.gamma) - 1 + (self.alpha - self.beta) * (self.t - 1)


# ---------------------------------------------------------------------------
# ring arithmetic modulo 2^64 and Phi_M
# ---------------------------------------------------------------------------
def fold_cyclic(P: NativeParams, c: np.ndarray) -> np.ndarray:
    """A polynomial modulo X^M - 1 (M coefficients) reduced modulo Phi_M."""
    assert c.shape[-1] == P.M
    N, Mt = P.N, P.Mt
    j = np.arange(N)
    return (c[..., :N] - c[..., N + (j % Mt)]).astype(U64)


def to_cyclic(P: NativeParams, full: np.ndarray) -> np.ndarray:
    """Any-length coefficient array folded modulo X^M - 1."""
    out = np.zeros(full.shape[:-1] + (P.M,), U64)
    for s in range(0, full.shape[-1], P.M):
        seg = full[..., s: s + P.M]
        out[..., : seg.shape[-1]] += seg
    return out


def mul(P: NativeParams, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a b mod (Phi_M, 2^64): the full convolution (library step, exact with uint64
    wrap-around), folded modulo X^M - 1, then modulo Phi_M."""
    full = np.convolve(a.astype(U64), b.astype(U64))
    return fold_cyclic(P, to_cyclic(P, full))


def mul_mono(P: NativeParams, a: np.ndarray, e: int) -> np.ndarray:
    """X^e a."""
    c = np.zeros(a.shape[:-1] + (P.M,), U64)
    c[..., (np.arange(P.N) + e) % P.M] = a
    return fold_cyclic(P, c)


def automorphism(P: NativeParams, a: np.ndarray, d: int) -> np.ndarray:
    """a(X^d) for a unit d modulo M."""
    assert np.gcd(d, P.M) == 1
    c = np.zeros(a.shape[:-1] + (P.M,), U64)
    c[..., (d * np.arange(P.N)) % P.M] = a
    return fold_cyclic(P, c)


def signed(x: np.ndarray) -> np.ndarray:
    return x.astype(U64).view(np.int64)


def from_signed(x) -> np.ndarray:
    return np.asarray(x, np.int64).view(U64)


# ---------------------------------------------------------------------------
# client: keys, encryption, decryption
# ---------------------------------------------------------------------------
class NativeClient:
    def __init__(self, P: NativeParams, seed: int):
        self.P = P
        self.rng = np.random.default_rng(seed)
        self.s = from_signed(self.rng.integers(-1, 2, P.N))

    def _err(self, shape):
        e = np.clip(np.round(self.rng.normal(0.0, self.P.sigma, shape)), -6 * self.P.sigma, 6 * self.P.sigma)
        return from_signed(e.astype(np.int64))

    def encrypt_torus(self, mu: np.ndarray) -> np.ndarray:
        """(a, b) with b = s a + mu + e; returns [2][N]."""
        P = self.P
        a = self.rng.integers(0, 2 ** 64, P.N, dtype=U64, endpoint=False)
        b = (mul(P, self.s, a) + mu.astype(U64) + self._err(P.N)).astype(U64)
        return np.stack([a, b])

    def encode(self, m) -> np.ndarray:
        """Message m (integers mod p, N coefficients) as torus values m 2^64 / p."""
        return (np.asarray(m, np.int64).astype(U64) % U64(self.P.p)) << U64(64 - self.P.log_p)

    def encrypt(self, m) -> np.ndarray:
        return self.encrypt_torus(self.encode(m))

    def phase(self, ct: np.ndarray) -> np.ndarray:
        return (ct[1] - mul(self.P, self.s, ct[0])).astype(U64)

    def decode(self, ph: np.ndarray) -> np.ndarray:
        """round(p ph / 2^64) mod p."""
        sh = U64(64 - self.P.log_p)
        return (((ph + (U64(1) << (sh - U64(1)))) >> sh) & U64(self.P.p - 1)).astype(np.int64)

    def decrypt(self, ct: np.ndarray) -> np.ndarray:
        return self.decode(self.phase(ct))

    def ksk(self, d: int) -> np.ndarray:
        """Key for sigma_d: the l encryptions of s(X^d) g_i, g_i = round(2^64 / D^i),
        [l][2][N]."""
        P = self.P
        sd = automorphism(P, self.s, d)
        return np.stack([self.encrypt_torus((sd * U64(P.gadget(i) % 2 ** 64)).astype(U64)) for i in range(1, P.l + 1)])

    def keyset(self) -> dict:
        """Keys of every Galois element the packing uses."""
        return {d: self.ksk(d) for d in self.P.taus()}

    def encrypt_powers(self, m) -> np.ndarray:
        """Encryptions of m(X^d) for the level-gamma exponents d, [n_pow][2][N]."""
        P = self.P
        mu = self.encode(m)
        return np.stack([self.encrypt_torus(automorphism(P, mu, d)) for d in P.powers()])


# ---------------------------------------------------------------------------
# server
# ---------------------------------------------------------------------------
def decompose(P: NativeParams, a: np.ndarray) -> np.ndarray:
    """Balanced gadget digits of a: a / 2^64 ~ sum_{i=1..l} d_i / D^i with d_i in
    [-D/2, D/2); returns int64 [l][...] (i = 1 first).  a / 2^64 is first rounded to a
    multiple of 1 / D^l: top = floor((a D^l + 2^63) / 2^64) (for D = 2^log_d, the top
    l log_d bits of a rounded); a carry out of the top digit is dropped (the torus
    wraps)."""
    D, l = P.D, P.l
    if P.base:
        Dl = D ** l
        flat = [(int(x) * Dl + (1 << 63)) >> 64 for x in np.asarray(a, U64).ravel()]
        top = np.array(flat, dtype=np.int64).reshape(np.shape(a))  # <= D^l < 2^63
    else:
        sh = 64 - P.log_d * l
        top = ((a.astype(U64) + (U64(1) << U64(sh - 1))) >> U64(sh)).astype(np.int64)  # < 2^(l log_d)
    digs = []
    for _ in range(l):  # least significant digit first
        d = top % D
        top = top // D
        neg = d >= D // 2
        d = np.where(neg, d - D, d)
        top = top + neg
        digs.append(d)
    return np.stack(digs[::-1])


def key_switch(P: NativeParams, ct: np.ndarray, key: np.ndarray) -> np.ndarray:
    """A ciphertext under s(X^d) to one under s with the key of sigma_d."""
    digs = decompose(P, ct[0])
    a = np.zeros(P.N, U64)
    b = ct[1].astype(U64).copy()
    for i in range(P.l):
        di = from_signed(digs[i])
        a = (a - mul(P, di, key[i][0])).astype(U64)
        b = (b - mul(P, di, key[i][1])).astype(U64)
    return np.stack([a, b])


def apply_galois(P: NativeParams, ct: np.ndarray, d: int, keys: dict) -> np.ndarray:
    """sigma_d of the encrypted message, under s again (one key switch)."""
    return key_switch(P, automorphism(P, ct, d), keys[d])


def extract(P: NativeParams, pows: np.ndarray) -> np.ndarray:
    """Rows E_i, i < N, of one chunk from the encryptions of its powers ([n_pow][2][N]):
    E_i = u sum_d ct_d (X^(d (M - i)) - X^(d (M/t - r))), r = i mod M/t.  [N][2][N]."""
    ds = P.powers()
    u = U64(P.u())
    out = np.zeros((P.N, 2, P.N), U64)
    for i in range(P.N):
        r = i % P.Mt
        acc = np.zeros((2, P.N), U64)
        for ct, d in zip(pows, ds):
            acc = (acc + mul_mono(P, ct, (d * (P.M - i)) % P.M) - mul_mono(P, ct, (d * (P.Mt - r)) % P.M)).astype(U64)
        out[i] = (acc * u).astype(U64)
    return out


def linear_rows(W: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """F_o = sum_i W[o][i] E_i mod 2^64 (W integer [n_out][n_in], rows [n_in][2][N])."""
    Wu = from_signed(np.asarray(W, np.int64))
    out = np.zeros((Wu.shape[0],) + rows.shape[1:], U64)
    for o in range(Wu.shape[0]):
        for i in np.nonzero(Wu[o])[0]:
            out[o] = (out[o] + Wu[o, i] * rows[i]).astype(U64)
    return out


def conv_matrix(c_in: int, c_out: int, h: int, w: int, k: int, stride: int, wts: np.ndarray) -> np.ndarray:
    """The integer matrix of a convolution over channels-last flattened inputs (index
    (y w + x) c_in + ci), zero padding k // 2: row (position p = y' w' + x', channel co),
    w' = (w - 1) // stride + 1, holds wts[co][ci][dy][dx] at the window's inputs (the
    paper's remark that a convolution is a matrix-vector product with its Toeplitz
    matrix, Sec. 4.4)."""
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    W = np.zeros((ho * wo * c_out, h * w * c_in), np.int64)
    for yo in range(ho):
        for xo in range(wo):
            for co in range(c_out):
                r = (yo * wo + xo) * c_out + co
                for dy in range(k):
                    for dx in range(k):
                        y, x = stride * yo + dy - k // 2, stride * xo + dx - k // 2
                        if 0 <= y < h and 0 <= x < w:
                            for ci in range(c_in):
                                W[r, (y * w + x) * c_in + ci] += wts[co, ci, dy, dx]
    return W


def pack(P: NativeParams, rows: np.ndarray, keys: dict, count: list | None = None) -> np.ndarray:
    """Fast packing of phi(t^beta) rows (fewer are zero-padded) into one ciphertext of
    sum_o y_o X^(o M / t^beta).  `count`, if given, gets the number of key switches."""
    t, M = P.t, P.M
    n = P.n_pack
    assert rows.shape[0] <= n
    F = np.zeros((n, 2, P.N), U64)
    F[: rows.shape[0]] = rows
    T = t ** (P.beta - P.gamma)
    phig = (t - 1) * t ** (P.gamma - 1)
    ks = 0
    cur = []
    for e in range(T):
        leaf = np.zeros((2, P.N), U64)
        for j in range(phig):
            leaf = (leaf + mul_mono(P, F[e + j * T], j * M // t ** P.gamma)).astype(U64)
        cur.append(leaf)
    for i in range(P.gamma, P.beta):
        th, tau = M // t ** (i + 1), (1 + t ** i) % M
        step = len(cur) // t
        nxt = []
        for r in range(step):
            ys = [cur[r + k * step] for k in range(t)]
            v = []
            for m in range(t):
                acc = np.zeros((2, P.N), U64)
                for k in range(t):
                    acc = (acc + mul_mono(P, ys[k], (k * (th - m * P.Mt)) % M)).astype(U64)
                v.append(acc)
            S = v[t - 1]
            for m in range(t - 2, -1, -1):
                S = (v[m] + apply_galois(P, S, tau, keys)).astype(U64)
                ks += 1
            nxt.append(S)
        cur = nxt
    Pk = cur[0]
    for j in range(P.alpha - 1, P.beta - 1, -1):
        tau = (1 + t ** j) % M
        S = Pk
        for _ in range(t - 1):
            S = (Pk + apply_galois(P, S, tau, keys)).astype(U64)
            ks += 1
        Pk = S
    if count is not None:
        count.append(ks)
    return Pk


def unpack_positions(P: NativeParams) -> np.ndarray:
    """Coefficient index of packed output o: o M / t^beta."""
    return np.arange(P.n_pack) * (P.M // P.t ** P.beta)


def server_layer(P: NativeParams, chunks: np.ndarray, W: np.ndarray, keys: dict, perm=None) -> np.ndarray:
    """The whole server round: extraction of every chunk ([n_chunks][n_pow][2][N]), the
    integer layer W on the rows (E = n_chunks N inputs, rows beyond W's columns unused),
    the shuffle (outputs reordered: row o of the result is output perm[o]) and the
    packing; returns [n_packs][2][N]."""
    rows = np.concatenate([extract(P, c) for c in chunks])[: W.shape[1]]
    Wp = np.asarray(W)[perm] if perm is not None else np.asarray(W)
    F = linear_rows(Wp, rows)
    n = P.n_pack
    return np.stack([pack(P, F[g: g + n], keys) for g in range(0, F.shape[0], n)])
