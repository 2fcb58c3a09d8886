"""Python driver of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It loads ``libckks_oracle.so`` (built from
``ckks_oracle.c`` with gcc) and adds the plaintext-side pieces that are
plain numpy:

  * CKKS encode/decode (Cheon-Kim-Kim-Song 2017): the canonical embedding
    with slot j at zeta^(5^j), zeta = exp(i pi/N), computed with numpy's FFT
    (a library FFT as one step) and pinned by the tests to the defining sums
    in ``ckks_oracle.c``;
  * the diagonal (Halevi-Shoup) and multiplexed-convolution schedules, i.e.
    which slot vectors get encoded and which rotations are applied;
  * the permutation folding W' = P_out W P_in^T of the shuffle / unshuffle
    steps (paper Sec. 4.4: the server unshuffles the previous round's
    permutation, runs the linear layer, and shuffles its output);
  * FP64 plaintext reference layers (paper Sec. 5: a fully connected layer
    or a convolution is a matrix-vector product).

It shares no code with the HIP library and never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "libckks_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent limbs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        u64, i64, i32, sz = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
        p = ctypes.c_void_p
        sig = {
            "or_mulmod": (u64, [u64, u64, u64]),
            "or_powmod": (u64, [u64, u64, u64]),
            "or_invmod": (u64, [u64, u64]),
            "or_is_prime": (i32, [u64]),
            "or_gen_primes": (i32, [i32, i32, i32, p]),
            "or_min_root": (u64, [u64, i32]),
            "or_ntt_naive": (None, [p, p, i32, u64, u64]),
            "or_ntt_naive_at": (u64, [p, sz, i32, u64, u64]),
            "or_intt_naive": (None, [p, p, i32, u64, u64]),
            "or_set_schoolbook": (None, [i32]),
            "or_polymul_schoolbook": (None, [p, p, p, i32, u64]),
            "or_polymul_fast": (None, [p, p, p, i32, u64]),
            "or_polymul_at": (u64, [p, p, sz, i32, u64]),
            "or_automorph": (None, [p, p, i32, u64, u64]),
            "or_modup": (None, [p, i32, i32, i32, i32, i32, p, p]),
            "or_moddown": (None, [p, i32, i32, i32, i32, i32, p, p]),
            "or_keyswitch": (None, [p, i32, p, i32, i32, i32, i32, p, p]),
            "or_rotate": (None, [p, i32, u64, p, i32, i32, i32, i32, p, p]),
            "or_ks_inner_at": (None, [p, i32, p, sz, i32, i32, i32, i32, p, p]),
            "or_moddown_at": (None, [p, i32, i32, i32, i32, i32, p, p]),
            "or_rescale": (None, [p, i32, i32, p, p]),
            "or_mul_pt": (None, [p, p, i32, i32, p, p]),
            "or_galois_of": (u64, [i64, i32]),
            "or_linear": (i32, [p, i32, i32, i32, p, i32, p, p, i32, i32, p, i32, p, i32, i32, i32, i32, p, p]),
            "or_linear_dh": (i32, [p, i32, i32, i32, p, i32, p, p, i32, i32, p, i32, p, i32, i32, i32, i32, p, p]),
            "or_encrypt": (None, [p, p, p, p, i32, i32, p, p]),
            "or_decrypt": (None, [p, p, i32, i32, p, p]),
            "or_keygen_galois": (None, [p, u64, p, p, i32, i32, i32, i32, p, p]),
            "or_crt_centered": (None, [p, i32, i32, p, p]),
            "or_encode_direct": (None, [p, p, i32, ctypes.c_double, p]),
            "or_decode_direct": (None, [p, i32, ctypes.c_double, p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
def gen_primes(log_n: int, bits: int, count: int) -> list[int]:
    out = np.zeros(count, np.uint64)
    got = lib().or_gen_primes(log_n, bits, count, _ptr(out))
    if got != count:
        raise ValueError("not enough primes")
    return [int(v) for v in out]


@dataclass
class Params:
    """RNS-CKKS parameters: N = 2^log_n, L primes q (descending), K special primes p."""

    log_n: int
    q: list
    p: list
    dnum: int
    scale: float = 2.0 ** 40
    mods_arr: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.mods_arr = _u64(list(self.q) + list(self.p))

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def S(self):
        return self.N // 2

    @property
    def L(self):
        return len(self.q)

    @property
    def K(self):
        return len(self.p)

    @property
    def alpha(self):
        return -(-self.L // self.dnum)

    def beta(self, level: int) -> int:
        return -(-level // self.alpha)

    @property
    def mods(self):
        return list(self.q) + list(self.p)


def make_params(log_n: int, L: int, K: int, dnum: int, bits: int, scale: float) -> Params:
    """Prime choice: scan down from 2^bits over q = 1 (mod 2N); the first K primes
    found are the special primes p, the next L are q_0 > q_1 > ... ."""
    pr = gen_primes(log_n, bits, K + L)
    return Params(log_n=log_n, q=pr[K:], p=pr[:K], dnum=dnum, scale=scale)


def galois_of(r: int, log_n: int) -> int:
    """Galois element of a left slot rotation by r: 5^(r mod N/2) mod 2N."""
    return int(lib().or_galois_of(int(r), log_n))


def min_root(q: int, log_n: int) -> int:
    return int(lib().or_min_root(q, log_n))


# --------------------------------------------------------------------------
# ring level
# --------------------------------------------------------------------------
def ntt_naive(a, log_n, q):
    a = _u64(a); out = np.zeros_like(a)
    lib().or_ntt_naive(_ptr(a), _ptr(out), log_n, q, min_root(q, log_n))
    return out


def ntt_naive_at(a, k, log_n, q, psi=None):
    a = _u64(a)
    return int(lib().or_ntt_naive_at(_ptr(a), int(k), log_n, q, psi or min_root(q, log_n)))


def intt_naive(A, log_n, q):
    A = _u64(A); out = np.zeros_like(A)
    lib().or_intt_naive(_ptr(A), _ptr(out), log_n, q, min_root(q, log_n))
    return out


def polymul_schoolbook(a, b, log_n, q):
    a, b = _u64(a), _u64(b); out = np.zeros_like(a)
    lib().or_polymul_schoolbook(_ptr(a), _ptr(b), _ptr(out), log_n, q)
    return out


def polymul_fast(a, b, log_n, q):
    a, b = _u64(a), _u64(b); out = np.zeros_like(a)
    lib().or_polymul_fast(_ptr(a), _ptr(b), _ptr(out), log_n, q)
    return out


def polymul_at(a, b, k, log_n, q):
    a, b = _u64(a), _u64(b)
    return int(lib().or_polymul_at(_ptr(a), _ptr(b), int(k), log_n, q))


def set_schoolbook(on: bool):
    lib().or_set_schoolbook(1 if on else 0)


def automorph(a, g, log_n, q):
    a = _u64(a); out = np.zeros_like(a)
    lib().or_automorph(_ptr(a), _ptr(out), log_n, int(g), q)
    return out


def automorph_limbs(x, g, log_n, mods):
    """Apply sigma_g to every limb of x [..., l, N]; limb i uses mods[i]."""
    x = _u64(x)
    out = np.empty_like(x)
    flat_in = x.reshape(-1, x.shape[-2], x.shape[-1])
    flat_out = out.reshape(flat_in.shape)
    for t in range(flat_in.shape[0]):
        for i in range(flat_in.shape[1]):
            flat_out[t, i] = automorph(flat_in[t, i], g, log_n, int(mods[i]))
    return out


# --------------------------------------------------------------------------
# key switching, rescale, products
# --------------------------------------------------------------------------
def modup(prm: Params, x, level):
    x = _u64(x)
    out = np.zeros((prm.beta(level), level + prm.K, prm.N), np.uint64)
    lib().or_modup(_ptr(x), level, prm.log_n, prm.L, prm.K, prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    return out


def moddown(prm: Params, u, level):
    u = _u64(u)
    out = np.zeros((level, prm.N), np.uint64)
    lib().or_moddown(_ptr(u), level, prm.log_n, prm.L, prm.K, prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    return out


def keyswitch(prm: Params, d, evk, level):
    d, evk = _u64(d), _u64(evk)
    out = np.zeros((2, level, prm.N), np.uint64)
    lib().or_keyswitch(_ptr(d), level, _ptr(evk), prm.log_n, prm.L, prm.K, prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    return out


def ks_inner_at(prm: Params, d, evk, level, k):
    d, evk = _u64(d), _u64(evk)
    out = np.zeros((2, level + prm.K), np.uint64)
    lib().or_ks_inner_at(_ptr(d), level, _ptr(evk), int(k), prm.log_n, prm.L, prm.K, prm.dnum,
                         _ptr(prm.mods_arr), _ptr(out))
    return out


def moddown_at(prm: Params, u_col, level):
    u_col = _u64(u_col)
    out = np.zeros(level, np.uint64)
    lib().or_moddown_at(_ptr(u_col), level, prm.log_n, prm.L, prm.K, prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    return out


def rotate(prm: Params, ct, g, evk, level):
    ct, evk = _u64(ct), _u64(evk)
    out = np.zeros((2, level, prm.N), np.uint64)
    lib().or_rotate(_ptr(ct), level, int(g), _ptr(evk), prm.log_n, prm.L, prm.K, prm.dnum,
                    _ptr(prm.mods_arr), _ptr(out))
    return out


def rescale(prm: Params, ct, level):
    ct = _u64(ct)
    out = np.zeros((2, level - 1, prm.N), np.uint64)
    lib().or_rescale(_ptr(ct), level, prm.log_n, _ptr(prm.mods_arr), _ptr(out))
    return out


def mul_pt(prm: Params, ct, pt, level):
    ct, pt = _u64(ct), _u64(pt[:level])
    out = np.zeros((2, level, prm.N), np.uint64)
    lib().or_mul_pt(_ptr(ct), _ptr(pt), level, prm.log_n, _ptr(prm.mods_arr), _ptr(out))
    return out


def linear(prm: Params, x, level, sched: "Schedule", pts, keys: "KeySet", hoist_moddown: bool = False):
    """Generic BSGS transform; x [n_in][2][level][N]; pts [n_out][n_in][G][B][pt_l + K][N]
    (rows: q_0..q_{pt_l-1} then p_0..p_{K-1}).  hoist_moddown selects the double-hoisted
    schedule (key-switch outputs kept in the extended basis)."""
    x = _u64(x)
    pts = _u64(pts)
    pt_l = pts.shape[-2] - prm.K
    assert pts.shape[:4] == (sched.n_out, sched.n_in, sched.G, sched.B) and pt_l >= level
    rb = np.ascontiguousarray(sched.rb, np.int64)
    gk = np.ascontiguousarray(sched.gk, np.int64)
    gal = np.ascontiguousarray(keys.galois, np.uint32)
    evk = keys.evk
    out = np.zeros((sched.n_out, 2, level, prm.N), np.uint64)
    if hoist_moddown:
        rc = lib().or_linear_dh(_ptr(x), sched.n_in, sched.n_out, sched.B, _ptr(rb), sched.G, _ptr(gk), _ptr(pts),
                                pt_l, level, _ptr(gal), len(keys.galois), _ptr(evk), prm.log_n, prm.L, prm.K,
                                prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    else:
        # the per-rotation schedule reads the q rows only
        pq = np.ascontiguousarray(pts[..., :pt_l, :])
        rc = lib().or_linear(_ptr(x), sched.n_in, sched.n_out, sched.B, _ptr(rb), sched.G, _ptr(gk), _ptr(pq),
                             pt_l, level, _ptr(gal), len(keys.galois), _ptr(evk), prm.log_n, prm.L, prm.K,
                             prm.dnum, _ptr(prm.mods_arr), _ptr(out))
    if rc != 0:
        raise KeyError("missing Galois key")
    return out


# --------------------------------------------------------------------------
# client side: keys, encryption, decryption (test-input construction only)
# --------------------------------------------------------------------------
@dataclass
class KeySet:
    galois: list
    evk: np.ndarray  # [n_keys][dnum][2][L+K][N]


def keygen_galois(prm: Params, s, g, a_rand, e):
    """a_rand [dnum][L+K][N] uniform per modulus; e [dnum][N] small ints."""
    s = np.ascontiguousarray(s, np.int8)
    a_rand = _u64(a_rand)
    e = np.ascontiguousarray(e, np.int64)
    out = np.zeros((prm.dnum, 2, prm.L + prm.K, prm.N), np.uint64)
    lib().or_keygen_galois(_ptr(s), int(g), _ptr(a_rand), _ptr(e), prm.log_n, prm.L, prm.K, prm.dnum,
                           _ptr(prm.mods_arr), _ptr(out))
    return out


def encrypt(prm: Params, m_rns, s, a, e, level):
    m_rns, a = _u64(m_rns[:level]), _u64(a[:level])
    s = np.ascontiguousarray(s, np.int8)
    e = np.ascontiguousarray(e, np.int64)
    out = np.zeros((2, level, prm.N), np.uint64)
    lib().or_encrypt(_ptr(m_rns), _ptr(s), _ptr(a), _ptr(e), level, prm.log_n, _ptr(prm.mods_arr), _ptr(out))
    return out


def decrypt(prm: Params, ct, s, level):
    ct = _u64(ct)
    s = np.ascontiguousarray(s, np.int8)
    out = np.zeros((level, prm.N), np.uint64)
    lib().or_decrypt(_ptr(ct), _ptr(s), level, prm.log_n, _ptr(prm.mods_arr), _ptr(out))
    return out


def crt_centered(prm: Params, m_rns, level) -> np.ndarray:
    """Centred CRT lift of [level][N] residues, as long double values."""
    m_rns = _u64(m_rns[:level])
    out = np.zeros(prm.N, np.longdouble)
    lib().or_crt_centered(_ptr(m_rns), level, prm.log_n, _ptr(prm.mods_arr), _ptr(out))
    return out


# --------------------------------------------------------------------------
# encode / decode
# --------------------------------------------------------------------------
def slot_exponents(log_n: int) -> np.ndarray:
    """5^j mod 2N for j < N/2 (int64)."""
    n2 = 2 << log_n
    out = np.empty(1 << (log_n - 1), np.int64)
    p = 1
    for j in range(out.size):
        out[j] = p
        p = p * 5 % n2
    return out


def encode_direct(z, log_n: int, delta: float) -> np.ndarray:
    """Defining-sum encode in long double (O(N^2)); integer coefficients."""
    z = np.asarray(z, np.complex128)
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    out = np.zeros(1 << log_n, np.int64)
    lib().or_encode_direct(_ptr(zr), _ptr(zi), log_n, float(delta), _ptr(out))
    return out


def decode_direct(m_centered, log_n: int, delta: float) -> np.ndarray:
    m = np.ascontiguousarray(m_centered, np.longdouble)
    s = 1 << (log_n - 1)
    zr, zi = np.zeros(s), np.zeros(s)
    lib().or_decode_direct(_ptr(m), log_n, float(delta), _ptr(zr), _ptr(zi))
    return zr + 1j * zi


def encode(z, log_n: int, delta: float) -> np.ndarray:
    """m_k = rint(Delta * (2/N) * Re(sum_j z_j zeta^(-5^j k))), ties to even.

    Over all odd exponents e (slot values z at 5^j, conj(z) at -5^j) this is
    (Delta/N) Re(sum_e Z_e zeta^(-e k)); with e = 2t+1 the sum is
    zeta^(-k) * sum_t Z_t w^(-t k), w = exp(2 pi i/N): a forward DFT."""
    n = 1 << log_n
    z = np.asarray(z, np.complex128)
    e = slot_exponents(log_n)
    Z = np.zeros(n, np.complex128)
    Z[(e - 1) // 2] = z
    Z[(2 * n - e - 1) // 2] = np.conj(z)
    k = np.arange(n)
    w = np.fft.fft(Z) * np.exp(-1j * np.pi * k / n)
    return np.rint(delta / n * w.real).astype(np.int64)


def decode(m_centered, log_n: int, delta: float) -> np.ndarray:
    """z_j = Delta^-1 sum_k m_k zeta^(5^j k); with 5^j = 2t+1 this is N * ifft(m zeta^k)[t]."""
    n = 1 << log_n
    m = np.asarray(m_centered, np.float64)
    k = np.arange(n)
    W = np.fft.ifft(m * np.exp(1j * np.pi * k / n)) * n
    e = slot_exponents(log_n)
    return W[(e - 1) // 2] / delta


def to_rns(m_int: np.ndarray, mods) -> np.ndarray:
    """Signed integers (int64) -> [len(mods)][N] residues."""
    m = np.asarray(m_int, np.int64)
    rows = []
    for q in mods:
        q = int(q)
        r = np.where(m >= 0, m.astype(np.uint64) % np.uint64(q),
                     (np.uint64(q) - ((-(m + 1)).astype(np.uint64) + np.uint64(1)) % np.uint64(q)) % np.uint64(q))
        rows.append(r.astype(np.uint64))
    return np.stack(rows)


def encode_rns(prm: Params, z, level: int, delta: float, ext: bool = False) -> np.ndarray:
    """Encoded slots as residues mod q_0..q_{level-1} (and p_0..p_{K-1} when ext)."""
    mods = prm.q[:level] + (prm.p if ext else [])
    return to_rns(encode(z, prm.log_n, delta), mods)


def decrypt_decode(prm: Params, ct, s, level: int, delta: float) -> np.ndarray:
    m = decrypt(prm, ct, s, level)
    return decode(crt_centered(prm, m, level).astype(np.float64), prm.log_n, delta)


# --------------------------------------------------------------------------
# linear-layer schedules (which rotations and which slot vectors)
# --------------------------------------------------------------------------
@dataclass
class Schedule:
    """y_o = sum_k rot_{gk[k]}( sum_i sum_b pt[o][i][k][b] * rot_{rb[b]}(x_i) )."""

    n_in: int
    n_out: int
    rb: list
    gk: list

    @property
    def B(self):
        return len(self.rb)

    @property
    def G(self):
        return len(self.gk)

    def rotations(self):
        return sorted({r for r in list(self.rb) + list(self.gk) if r != 0})


def fc_schedule(n: int, n1: int) -> Schedule:
    """Halevi-Shoup diagonal method, baby-step giant-step with n = n1 * n2
    (n1 = n: the plain method, one giant step)."""
    assert n % n1 == 0
    n2 = n // n1
    return Schedule(1, 1, list(range(n1)), [n1 * j for j in range(n2)])


def fold_permutations(W: np.ndarray, perm_out=None, perm_in=None) -> np.ndarray:
    """W'[t, u] = W[perm_out[t], perm_in[u]] (rows/cols unchanged when a perm is None).
    For a conv weight [C_out][C_in][kh][kw] the permutations act on channels."""
    Wp = W
    if perm_out is not None:
        Wp = Wp[np.asarray(perm_out)]
    if perm_in is not None:
        Wp = Wp[:, np.asarray(perm_in)]
    return Wp


def fc_slots(Wp: np.ndarray, n: int, n1: int, S: int) -> np.ndarray:
    """Plaintext slot vectors [1][1][n2][n1][S] for the FC schedule.

    W' (out_features x in_features) is zero-padded to n x n; diagonal i is
    d_i[s] = W'[s mod n, (s + i) mod n]; baby/giant entry (j, b) holds
    rot_{-n1 j}(d_{n1 j + b}) so that rot_{n1 j} brings it back in place."""
    Wn = np.zeros((n, n))
    Wn[: Wp.shape[0], : Wp.shape[1]] = Wp
    n2 = n // n1
    s = np.arange(S)
    out = np.zeros((1, 1, n2, n1, S))
    for j in range(n2):
        for b in range(n1):
            i = n1 * j + b
            d = Wn[s % n, (s + i) % n]
            out[0, 0, j, b] = np.roll(d, n1 * j)  # rot_{-n1 j}: out[s] = d[s - n1 j]
    return out


def fc_input_slots(x: np.ndarray, n: int, S: int) -> np.ndarray:
    """x (length <= n) zero-padded to n and replicated S/n times."""
    xn = np.zeros(n)
    xn[: x.size] = x
    return np.tile(xn, S // n)


def fc_output_from_slots(z: np.ndarray, out_features: int) -> np.ndarray:
    return np.asarray(z)[:out_features]


@dataclass
class ConvShape:
    c_in: int
    c_out: int
    h: int
    w: int
    k: int  # 1 or 3, stride 1, padding k // 2

    def per_ct(self, S: int) -> int:
        hw = self.h * self.w
        assert S % hw == 0
        return S // hw

    def n_in(self, S):
        return -(-self.c_in // self.per_ct(S))

    def n_out(self, S):
        return -(-self.c_out // self.per_ct(S))


def conv_schedule(cs: ConvShape, S: int, n1: int = 1) -> Schedule:
    """Multiplexed (channel-major) packing: slot s = c*H*W + h*W + w, c_ct = S/(H*W)
    channels per ciphertext.  The channel offsets k < c_ct split as k = k1 + n1 k2
    (baby-step giant-step over the channel rotation; n1 = 1: every channel offset a
    giant step).  Baby steps: channel offset k1 < n1 with each of the k*k spatial
    offsets (dy, dx) in row-major order, rotation k1*H*W + dy*W + dx.  Giant steps:
    rotation n1 k2 H*W."""
    c_ct = cs.per_ct(S)
    assert n1 >= 1 and c_ct % n1 == 0
    hw = cs.h * cs.w
    r = cs.k // 2
    offs = [0] if cs.k == 1 else [dy * cs.w + dx for dy in range(-r, r + 1) for dx in range(-r, r + 1)]
    rb = [k1 * hw + o for k1 in range(n1) for o in offs]
    gk = [n1 * k2 * hw for k2 in range(c_ct // n1)]
    return Schedule(cs.n_in(S), cs.n_out(S), rb, gk)


def conv_slots(Wp: np.ndarray, cs: ConvShape, S: int, n1: int = 1) -> np.ndarray:
    """Plaintext slot vectors [n_out][n_in][c_ct / n1][n1 k*k][S] for conv_schedule(cs, S, n1).

    With d_{k,(dy,dx)} the diagonal of channel offset k and spatial offset (dy, dx),
    at output slot s = co*HW + h*W + w of output ciphertext o,
    d[s] = W'[o c_ct + co, i c_ct + (co + k) mod c_ct, dy + r, dx + r]
           * [0 <= h + dy < H] * [0 <= w + dx < W]
    (zero where a channel index is past C_out / C_in), entry (o, i, k2, (k1, b)) is
    rot_{-n1 k2 H W}(d_{k1 + n1 k2, b}): the giant rotation by n1 k2 H W brings it back
    in place, and rot_{n1 k2 HW}(rot_{-n1 k2 HW}(d) * rot_{k1 HW + off}(x)) =
    d * rot_{k HW + off}(x)."""
    c_ct = cs.per_ct(S)
    assert n1 >= 1 and c_ct % n1 == 0
    hw = cs.h * cs.w
    n_in, n_out = cs.n_in(S), cs.n_out(S)
    r = cs.k // 2
    offs = [(dy, dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1)]
    s = np.arange(S)
    co = s // hw
    hh = (s % hw) // cs.w
    ww = s % cs.w
    n2 = c_ct // n1
    out = np.zeros((n_out, n_in, n2, n1 * len(offs), S))
    for o in range(n_out):
        co_g = o * c_ct + co
        for i in range(n_in):
            for k2 in range(n2):
                for k1 in range(n1):
                    k = k1 + n1 * k2
                    ci_g = i * c_ct + (co + k) % c_ct
                    valid_c = (co_g < cs.c_out) & (ci_g < cs.c_in)
                    for b, (dy, dx) in enumerate(offs):
                        valid = valid_c & (hh + dy >= 0) & (hh + dy < cs.h) & (ww + dx >= 0) & (ww + dx < cs.w)
                        d = np.zeros(S)
                        d[valid] = Wp[co_g[valid], ci_g[valid], dy + r, dx + r]
                        out[o, i, k2, k1 * len(offs) + b] = np.roll(d, n1 * k2 * hw)
    return out


def conv_input_slots(x: np.ndarray, cs: ConvShape, S: int) -> np.ndarray:
    """x [C_in][H][W] -> [n_in][S] channel-major slot vectors (zero-padded channels)."""
    c_ct = cs.per_ct(S)
    n_in = cs.n_in(S)
    buf = np.zeros((n_in * c_ct, cs.h, cs.w))
    buf[: cs.c_in] = x
    return buf.reshape(n_in, S)


def conv_output_from_slots(z: np.ndarray, cs: ConvShape, S: int) -> np.ndarray:
    """[n_out][S] slot vectors -> [C_out][H][W]."""
    z = np.asarray(z).reshape(-1, cs.h, cs.w)
    return z[: cs.c_out]


def conv_ref(Wp: np.ndarray, x: np.ndarray) -> np.ndarray:
    """FP64 'same' convolution, stride 1, zero padding k//2 (cross-correlation)."""
    c_out, c_in, k, _ = Wp.shape
    r = k // 2
    _, h, w = x.shape
    xp = np.zeros((c_in, h + 2 * r, w + 2 * r))
    xp[:, r:r + h, r:r + w] = x
    y = np.zeros((c_out, h, w))
    for dy in range(k):
        for dx in range(k):
            y += np.einsum("oc,chw->ohw", Wp[:, :, dy, dx], xp[:, dy:dy + h, dx:dx + w])
    return y
