"""The C ABI library: built, loadable without a GPU, and exporting exactly the
entry points that include/fhelin.h declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "fhelin.h")
LIB = os.path.join(ROOT, "paper_2509_01253_amd", "libfhelin.so")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(fhelin_\w+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for n in ["fhelin_ctx_create", "fhelin_keyset_load", "fhelin_pt_encode", "fhelin_plan_encode_weights",
              "fhelin_linear_apply", "fhelin_rescale", "fhelin_rotate", "fhelin_ntt", "fhelin_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2509_01253_amd.build)"
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = sorted({line.split()[-1] for line in out.splitlines() if " T " in line and "fhelin_" in line})
    assert exported == declared()


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.fhelin_status_string.restype = ctypes.c_char_p
    assert lib.fhelin_status_string(0) == b"ok"
    assert lib.fhelin_status_string(-4) == b"missing Galois key"


def test_prime_helper_matches_oracle():
    """The library's prime scan (host code, no GPU) and the oracle's agree."""
    from oracle import oracle as O
    lib = ctypes.CDLL(LIB)
    lib.fhelin_primes_generate.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_void_p]
    for log_n, bits, count in [(12, 36, 4), (15, 50, 10), (16, 50, 15)]:
        out = (ctypes.c_uint64 * count)()
        assert lib.fhelin_primes_generate(log_n, bits, count, ctypes.cast(out, ctypes.c_void_p)) == 0
        assert list(out) == O.gen_primes(log_n, bits, count)
    bad = (ctypes.c_uint64 * 1)()
    assert lib.fhelin_primes_generate(16, 10, 1, ctypes.cast(bad, ctypes.c_void_p)) == -1


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int32), ("n_q", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("dnum", ctypes.c_int32), ("q", ctypes.c_void_p), ("p", ctypes.c_void_p)]


def _create(lib, log_n, q, p, dnum):
    qa = (ctypes.c_uint64 * max(1, len(q)))(*q)
    pa = (ctypes.c_uint64 * max(1, len(p)))(*p)
    prm = _Params(log_n, len(q), len(p), dnum, ctypes.cast(qa, ctypes.c_void_p), ctypes.cast(pa, ctypes.c_void_p))
    out = ctypes.c_void_p()
    return lib.fhelin_ctx_create(ctypes.byref(prm), ctypes.byref(out)), out


def test_ctx_create_rejects_bad_parameters_on_the_host():
    """Parameter checks run before any HIP call (this machine has no GPU): each bad
    set returns its status and a message, and nothing is created."""
    from oracle import oracle as O
    lib = ctypes.CDLL(LIB)
    lib.fhelin_last_error.restype = ctypes.c_char_p
    pr = O.gen_primes(12, 50, 8)           # q = 1 mod 2^13, descending
    p, q = pr[:2], pr[2:8]
    bad = {
        "log_n": (9, q, p, 3, -2, b"log_n"),
        "dnum 0": (12, q, p, 0, -2, b"dnum"),
        "dnum > n_q": (12, q, p, 7, -2, b"dnum"),
        "not prime": (12, q[:5] + [q[5] + 2 * 8192], p, 3, -2, b"prime"),
        "not 1 mod 2N": (12, q[:5] + [pr[0] + 2], p, 3, -2, b"1 mod 2N"),
        "duplicate": (12, q[:5] + [q[0]], p, 3, -2, b"distinct"),
        "too large": (12, q[:5] + [(1 << 60) + 1], p, 3, -2, b"2^60"),
        "P too small": (12, q, p[:1], 2, -2, b"special modulus"),
        "no special prime": (12, q, [], 3, -2, b"n_p"),
        "too many digits' primes": (12, O.gen_primes(12, 50, 20)[2:20], p, 2, -2, b"digits"),
    }
    for name, (log_n, qq, pp, dnum, status, msg) in bad.items():
        rc, out = _create(lib, log_n, qq, pp, dnum)
        assert rc == status, name
        assert msg in lib.fhelin_last_error(), (name, lib.fhelin_last_error())
        assert not out.value, name
    assert lib.fhelin_ctx_create(None, None) == -1


def test_null_and_unknown_handles_rejected_without_a_gpu():
    """Destroy/release and layer calls take only handles the library handed out:
    null or foreign pointers are rejected with FHELIN_E_INVALID_ARG before anything
    is dereferenced."""
    lib = ctypes.CDLL(LIB)
    lib.fhelin_last_error.restype = ctypes.c_char_p
    fake = ctypes.create_string_buffer(4096)
    for fn in ("fhelin_ctx_destroy", "fhelin_keyset_release", "fhelin_ptset_release", "fhelin_plan_destroy",
               "fhelin_graph_destroy"):
        f = getattr(lib, fn)
        f.argtypes = [ctypes.c_void_p]
        assert f(None) == -1, fn
        assert f(ctypes.addressof(fake)) == -1, fn
        assert b"handle" in lib.fhelin_last_error()
    lib.fhelin_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.fhelin_graph_launch(ctypes.addressof(fake), None) == -1
    lib.fhelin_linear_apply.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int32, ctypes.c_void_p]
    assert lib.fhelin_linear_apply(ctypes.addressof(fake), ctypes.addressof(fake), None, ctypes.addressof(fake),
                                   None, None, 0, None) == -1
    assert b"context" in lib.fhelin_last_error()


class _NatPrm(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("t", "alpha", "gamma", "beta", "log_d", "l", "log_p", "engine", "base")]


def test_native_create_rejects_bad_parameters_on_the_host():
    """The paper's own pipeline checks its parameters before any device call: t an odd
    prime, M = t^alpha <= 8192, 1 <= gamma <= 2, gamma <= beta <= alpha - 1, the gadget
    and the message modulus in range; null and unknown handles are rejected."""
    lib = ctypes.CDLL(LIB)
    lib.fhelin_last_error.restype = ctypes.c_char_p
    lib.fhelin_native_create.argtypes = [ctypes.POINTER(_NatPrm), ctypes.POINTER(ctypes.c_void_p)]
    good = dict(t=3, alpha=7, gamma=1, beta=6, log_d=9, l=3, log_p=8, engine=0, base=0)
    bad = {"t even": dict(t=4), "t not prime": dict(t=9), "t = 2": dict(t=2), "alpha 1": dict(alpha=1),
           "M too large": dict(alpha=9), "gamma 0": dict(gamma=0), "gamma 3": dict(gamma=3, beta=5),
           "beta < gamma": dict(gamma=2, beta=1), "beta = alpha": dict(beta=7), "log_d 0": dict(log_d=0),
           "log_d 17": dict(log_d=17), "l 9": dict(l=9, log_d=4), "gadget 64 bits": dict(log_d=16, l=4),
           "log_p 0": dict(log_p=0), "log_p 32": dict(log_p=32), "engine 2": dict(engine=2),
           "odd base": dict(base=311), "base 2": dict(base=2), "base above 2^16": dict(base=65538, engine=1, l=2),
           "D^l >= 2^63": dict(base=310, l=8, engine=1), "int8 engine, base above 2^16": dict(base=65538, l=2)}
    for name, change in bad.items():
        out = ctypes.c_void_p()
        prm = _NatPrm(**{**good, **change})
        assert lib.fhelin_native_create(ctypes.byref(prm), ctypes.byref(out)) == -2, name
        assert not out.value, name
    # the paper's 16-bit set gadget passes the parameter checks on both engines (without
    # a GPU the call then fails at the device query, not as an unsupported parameter)
    lib.fhelin_native_destroy.argtypes = [ctypes.c_void_p]
    for eng in (0, 1):
        out = ctypes.c_void_p()
        prm = _NatPrm(**{**good, "t": 5, "alpha": 5, "beta": 4, "l": 4, "log_p": 16, "base": 310, "engine": eng})
        rc = lib.fhelin_native_create(ctypes.byref(prm), ctypes.byref(out))
        assert rc != -2, lib.fhelin_last_error()
        if rc == 0:
            assert lib.fhelin_native_destroy(out) == 0
    assert lib.fhelin_native_create(None, None) == -1
    fake = ctypes.create_string_buffer(4096)
    lib.fhelin_native_destroy.argtypes = [ctypes.c_void_p]
    assert lib.fhelin_native_destroy(None) == -1
    assert lib.fhelin_native_destroy(ctypes.addressof(fake)) == -1
    assert b"native" in lib.fhelin_last_error()


def test_issue_rate_probe_rejects_bad_arguments_on_the_host():
    """fhelin_diag_alu_rate checks the probe, the waves per SIMD and the round count
    before any device call (op 9 is the int8 matrix-core probe)."""
    lib = ctypes.CDLL(LIB)
    lib.fhelin_last_error.restype = ctypes.c_char_p
    d = ctypes.c_double
    lib.fhelin_diag_alu_rate.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(d),
                                         ctypes.POINTER(d), ctypes.POINTER(d)]
    for op, wps, iters in ((10, 2, 32), (-1, 2, 32), (9, 0, 32), (9, 9, 32), (9, 2, 31), (9, 2, 16), (5, 4, 1 << 25)):
        assert lib.fhelin_diag_alu_rate(op, wps, iters, None, None, None) == -1, (op, wps, iters)
    assert b"diag" in lib.fhelin_last_error()
