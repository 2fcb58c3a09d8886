"""The paper's own server pipeline on the GPU (RLWE over Z_{2^64}[X]/Phi_M): partial
trace extraction, the integer layer on the extracted rows with a folded shuffle, and
fast packing, through the C ABI, compared with the oracle element by element at every
stage, and the packed ciphertexts decrypted to the integer layer's outputs."""
import numpy as np
import pytest

from oracle import native_rlwe as R
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _csr(W):
    """CSR of an integer matrix: (row_ptr, col, val) as int32 arrays."""
    rows, cols = np.nonzero(W)
    row_ptr = np.zeros(W.shape[0] + 1, np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), W[rows, cols].astype(np.int32)


def _i32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def _conv_like(rng, n_out, n_in, nnz, mag):
    """Integer weights with nnz nonzeros per output (a convolution's row shape)."""
    W = np.zeros((n_out, n_in), np.int64)
    for o in range(n_out):
        idx = rng.choice(n_in, nnz, replace=False)
        W[o, idx] = rng.integers(-mag, mag, nnz)
    return W


def _run(F, P, chunks, W, perm, keys, engine=0):
    """GPU pipeline; returns (rows, F rows, packed) on the host."""
    import torch
    nt = F.fhelin_native_create(P.t, P.alpha, P.gamma, P.beta, P.log_d, P.l, P.log_p, engine, P.base)
    try:
        ksk = np.stack([keys[d] for d in P.taus()])
        F.fhelin_native_keys_load(nt, dev(ksk))
        x = dev(chunks)
        rows = torch.zeros((chunks.shape[0] * P.N, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_extract(nt, x, rows)
        rp, col, val = _csr(np.asarray(W)[perm])
        out = torch.zeros((W.shape[0], 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_linear(nt, _i32(rp), _i32(col), _i32(val), rows, out)
        n_packs = (W.shape[0] + P.n_pack - 1) // P.n_pack
        packed = torch.zeros((n_packs, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_pack(nt, out, packed)
        return host(rows), host(out), host(packed)
    finally:
        F.fhelin_native_destroy(nt)


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("t,alpha,gamma,beta", [(3, 4, 1, 3), (3, 4, 2, 3), (5, 3, 1, 2), (5, 3, 2, 2), (7, 2, 1, 1),
                                                (3, 5, 1, 2)])
def test_native_pipeline_bit_exact_small_rings(t, alpha, gamma, beta, engine):
    """Both key-switch engines (int8 matrix cores, 64-bit ALU) give the oracle's bits."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native t={t} alpha={alpha} gamma={gamma} beta={beta} engine={engine}", flush=True)
    P = R.NativeParams(t, alpha, gamma, beta, 9, 3, 8, 2.0 ** 28)
    cl = R.NativeClient(P, 100 + t * 10 + alpha)
    keys = cl.keyset()
    rng = np.random.default_rng(t * 100 + alpha * 10 + gamma)
    n_in = P.N + P.N // 3
    x = rng.integers(0, 16, n_in)
    chunks = []
    for c in range(2):
        m = np.zeros(P.N, np.int64)
        part = x[c * P.N: (c + 1) * P.N]
        m[: part.size] = part
        chunks.append(cl.encrypt_powers(m))
    chunks = np.stack(chunks)
    n_out = 2 * P.n_pack + 5  # two full packs and a partial one
    W = _conv_like(rng, n_out, n_in, min(24, n_in), 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, engine)
    want_rows = np.concatenate([R.extract(P, c) for c in chunks])
    assert np.array_equal(rows, want_rows)
    want_F = R.linear_rows(W[perm], want_rows[:n_in])
    assert np.array_equal(Fo, want_F)
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        want = R.pack(P, want_F[g * P.n_pack: (g + 1) * P.n_pack], keys)
        assert np.array_equal(packed[g], want), g
        dec = cl.decrypt(packed[g])
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        exp = np.zeros(P.N, np.int64)
        exp[pos[: seg.size]] = seg
        assert np.array_equal(dec, exp), g


@pytest.mark.parametrize("t,alpha,gamma,n_chunks", [(11, 3, 1, 2), (13, 3, 1, 2), (7, 3, 2, 2), (3, 8, 1, 1)])
def test_native_extract_rings_outside_lds(t, alpha, gamma, n_chunks):
    """Extraction where the chunk's powers do not fit LDS whole: rings with M <= 4096
    streamed power by power (t = 11: four workgroups of rows per residue r, the last
    with one row; t = 13: four of three; M = 7^3 at gamma = 2: 42 powers, two of
    three) and M = 3^8 > 4096 on the gather kernel; uniform 64-bit inputs (extraction
    is linear over Z_{2^64}), every row element by element."""
    from paper_2509_01253_amd import fhelin as F
    import torch
    print(f"native extract t={t} alpha={alpha} gamma={gamma} chunks={n_chunks}", flush=True)
    P = R.NativeParams(t, alpha, gamma, alpha - 1, 9, 3, 8, 2.0 ** 28)
    rng = np.random.default_rng(1300 + t * 10 + alpha + gamma)
    pows = rng.integers(0, 2 ** 64, (n_chunks, len(P.powers()), 2, P.N), dtype=np.uint64)
    nt = F.fhelin_native_create(P.t, P.alpha, P.gamma, P.beta, P.log_d, P.l, P.log_p, 0, P.base)
    try:
        rows = torch.zeros((n_chunks * P.N, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_extract(nt, dev(pows), rows)
        got = host(rows)
    finally:
        F.fhelin_native_destroy(nt)
    for c in range(n_chunks):
        assert np.array_equal(got[c * P.N: (c + 1) * P.N], R.extract(P, pows[c])), c


@pytest.mark.parametrize("t,alpha,gamma,beta,packs,log_d,l", [(3, 5, 1, 4, 30, 9, 3), (3, 5, 2, 4, 90, 9, 3),
                                                               (5, 4, 1, 3, 60, 9, 3), (7, 3, 1, 2, 260, 9, 3),
                                                               (5, 4, 1, 3, 60, 16, 2)])
def test_native_pack_many_packs(t, alpha, gamma, beta, packs, log_d, l):
    """Packing enough outputs that a merge level has a workgroup per compute unit for
    every (sub-pack, pack) pair, where the merge terms stage their sub-packs in LDS
    (the smaller levels of the same call keep the gather kernel; key switches with two
    digit pieces at D = 2^9, three at 2^16): uniform 64-bit layer outputs, the last
    pack partial, every packed ciphertext element by element against the oracle."""
    from paper_2509_01253_amd import fhelin as F
    import torch
    print(f"native pack t={t} alpha={alpha} gamma={gamma} beta={beta} packs={packs} log_d={log_d}", flush=True)
    P = R.NativeParams(t, alpha, gamma, beta, log_d, l, 8 if log_d == 9 else 12, 2.0 ** 28 if log_d == 9 else 2.0 ** 13)
    keys = R.NativeClient(P, 1400 + t * 10 + alpha + gamma).keyset()
    rng = np.random.default_rng(1410 + t * 10 + alpha + gamma)
    n_out = packs * P.n_pack - 7
    rows = rng.integers(0, 2 ** 64, (n_out, 2, P.N), dtype=np.uint64)
    nt = F.fhelin_native_create(P.t, P.alpha, P.gamma, P.beta, P.log_d, P.l, P.log_p, 0, P.base)
    try:
        F.fhelin_native_keys_load(nt, dev(np.stack([keys[d] for d in P.taus()])))
        packed = torch.zeros((packs, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_pack(nt, dev(rows), packed)
        got = host(packed)
    finally:
        F.fhelin_native_destroy(nt)
    for g in range(packs):
        assert np.array_equal(got[g], R.pack(P, rows[g * P.n_pack: (g + 1) * P.n_pack], keys)), g


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("gamma", [1, 2])
def test_native_pipeline_paper_8bit_set(gamma, engine):
    """The paper's 8-bit parameter set (M = 3^7, D = 512, l = 3, p = 2^8) with packs of
    phi(3^6) = 486 outputs: a convolution-shaped layer (144 weights of 4 bits per
    output) over two chunks; rows and layer outputs compared on sampled rows, every
    packed ciphertext element by element, and the decryptions equal to the layer."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native 3^7 gamma={gamma} engine={engine}", flush=True)
    P = R.NativeParams(3, 7, gamma, 6, 9, 3, 8, 2.0 ** 28)
    cl = R.NativeClient(P, 700 + gamma)
    keys = cl.keyset()
    rng = np.random.default_rng(710 + gamma)
    n_in = 2 * P.N
    x = rng.integers(0, 16, n_in)
    chunks = np.stack([cl.encrypt_powers(x[c * P.N: (c + 1) * P.N]) for c in range(2)])
    n_out = 2 * P.n_pack + 7
    W = _conv_like(rng, n_out, n_in, 144, 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, engine)
    for c in range(2):
        want = R.extract(P, chunks[c])
        sel = rng.choice(P.N, 40, replace=False)
        assert np.array_equal(rows[c * P.N + sel], want[sel]), c
    sel = rng.choice(n_out, 30, replace=False)
    assert np.array_equal(Fo[sel], R.linear_rows(W[perm][sel], rows))
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        want = R.pack(P, Fo[g * P.n_pack: (g + 1) * P.n_pack], keys)
        assert np.array_equal(packed[g], want), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(packed[g])[pos[: seg.size]], seg), g


@pytest.mark.parametrize("gamma,engine", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_native_pipeline_paper_12bit_set(gamma, engine):
    """The paper's 12-bit set (M = 7^4, N = 2058, D = 2^16, l = 2, p = 2^12, noise
    2^-51) on both engines (the int8 matrix cores split its digits into three pieces), packs of
    phi(7^3) = 294 outputs: a convolution-shaped layer (144 weights of 4 bits per
    output) over two chunks (one at gamma = 2, whose 42 powers make the oracle's
    extraction slow); rows and layer outputs compared on sampled rows, every packed
    ciphertext element by element, and the decryptions equal to the layer mod p."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native 7^4 gamma={gamma} engine={engine}", flush=True)
    P = R.NativeParams(7, 4, gamma, 3, 16, 2, 12, 2.0 ** 13)
    cl = R.NativeClient(P, 1200 + gamma)
    keys = cl.keyset()
    rng = np.random.default_rng(1210 + gamma)
    n_chunks = 2 if gamma == 1 else 1
    n_in = n_chunks * P.N
    x = rng.integers(0, 16, n_in)
    chunks = np.stack([cl.encrypt_powers(x[c * P.N: (c + 1) * P.N]) for c in range(n_chunks)])
    n_out = 2 * P.n_pack + 7
    W = _conv_like(rng, n_out, n_in, 144, 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, engine)
    for c in range(n_chunks):
        want = R.extract(P, chunks[c])
        sel = rng.choice(P.N, 40, replace=False)
        assert np.array_equal(rows[c * P.N + sel], want[sel]), c
    sel = rng.choice(n_out, 30, replace=False)
    assert np.array_equal(Fo[sel], R.linear_rows(W[perm][sel], rows))
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        want = R.pack(P, Fo[g * P.n_pack: (g + 1) * P.n_pack], keys)
        assert np.array_equal(packed[g], want), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(packed[g])[pos[: seg.size]], seg), g


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("t,alpha,gamma,beta", [(5, 3, 1, 2), (3, 4, 2, 3)])
def test_native_pipeline_base_310_small_rings(t, alpha, gamma, beta, engine):
    """The paper's 16-bit-set gadget (base 310, depth 4, p = 2^16) on small rings,
    both key-switch engines: rows, layer outputs and every packed ciphertext element
    by element against the oracle, decryptions equal to the layer."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native base 310 t={t} alpha={alpha} gamma={gamma} beta={beta} engine={engine}", flush=True)
    P = R.NativeParams(t, alpha, gamma, beta, 0, 4, 16, 2.0 ** 13, base=310)
    cl = R.NativeClient(P, 500 + t * 10 + alpha)
    keys = cl.keyset()
    rng = np.random.default_rng(510 + t * 10 + gamma)
    n_in = P.N + P.N // 3
    x = rng.integers(0, 16, n_in)
    chunks = []
    for c in range(2):
        m = np.zeros(P.N, np.int64)
        part = x[c * P.N: (c + 1) * P.N]
        m[: part.size] = part
        chunks.append(cl.encrypt_powers(m))
    chunks = np.stack(chunks)
    n_out = 2 * P.n_pack + 5
    W = _conv_like(rng, n_out, n_in, min(24, n_in), 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, engine)
    want_rows = np.concatenate([R.extract(P, c) for c in chunks])
    assert np.array_equal(rows, want_rows)
    want_F = R.linear_rows(W[perm], want_rows[:n_in])
    assert np.array_equal(Fo, want_F)
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        assert np.array_equal(packed[g], R.pack(P, want_F[g * P.n_pack: (g + 1) * P.n_pack], keys)), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(packed[g])[pos[: seg.size]], seg), g


@pytest.mark.parametrize("t,alpha,gamma,beta,log_d,l,base", [(3, 4, 1, 3, 12, 2, 0), (5, 3, 2, 2, 0, 2, 1000),
                                                              (3, 4, 2, 3, 16, 2, 0)])
def test_native_three_piece_digits_small_rings(t, alpha, gamma, beta, log_d, l, base):
    """Gadget bases above 2^9 (2^12, 1000, 2^16) on small rings: the int8 engine's
    three-piece digits against the oracle (rows, layer outputs, every packed ciphertext
    element by element) and the ALU engine giving the same bits."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native three pieces t={t} alpha={alpha} gamma={gamma} log_d={log_d} l={l} base={base}", flush=True)
    P = R.NativeParams(t, alpha, gamma, beta, log_d, l, 12, 2.0 ** 13, base=base)
    cl = R.NativeClient(P, 900 + t * 10 + alpha + base % 97)
    keys = cl.keyset()
    rng = np.random.default_rng(910 + t * 10 + gamma)
    n_in = P.N + P.N // 3
    x = rng.integers(0, 16, n_in)
    chunks = []
    for c in range(2):
        m = np.zeros(P.N, np.int64)
        part = x[c * P.N: (c + 1) * P.N]
        m[: part.size] = part
        chunks.append(cl.encrypt_powers(m))
    chunks = np.stack(chunks)
    n_out = 2 * P.n_pack + 5
    W = _conv_like(rng, n_out, n_in, min(24, n_in), 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, 0)
    want_rows = np.concatenate([R.extract(P, c) for c in chunks])
    assert np.array_equal(rows, want_rows)
    want_F = R.linear_rows(W[perm], want_rows[:n_in])
    assert np.array_equal(Fo, want_F)
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        assert np.array_equal(packed[g], R.pack(P, want_F[g * P.n_pack: (g + 1) * P.n_pack], keys)), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(packed[g])[pos[: seg.size]], seg), g
    assert np.array_equal(_run(F, P, chunks, W, perm, keys, 1)[2], packed)


@pytest.mark.parametrize("gamma,engine", [(1, 0), (2, 1)])
def test_native_pipeline_paper_16bit_set(gamma, engine):
    """The paper's 16-bit set (M = 5^5, N = 2500, D = 310, l = 4, p = 2^16, noise
    2^-51), packs of phi(5^4) = 500 outputs; gamma = 1 on the int8 matrix cores
    (digits of base 310 fit the 4/5-bit split), gamma = 2 on the 64-bit ALU engine
    (one chunk: its 20 powers make the oracle's extraction slow).  Sampled rows and
    layer outputs, every packed ciphertext element by element, decryptions equal to
    the layer mod p."""
    from paper_2509_01253_amd import fhelin as F
    print(f"native 5^5 base 310 gamma={gamma} engine={engine}", flush=True)
    P = R.NativeParams(5, 5, gamma, 4, 0, 4, 16, 2.0 ** 13, base=310)
    cl = R.NativeClient(P, 1600 + gamma)
    keys = cl.keyset()
    rng = np.random.default_rng(1610 + gamma)
    n_chunks = 2 if gamma == 1 else 1
    n_in = n_chunks * P.N
    x = rng.integers(0, 16, n_in)
    chunks = np.stack([cl.encrypt_powers(x[c * P.N: (c + 1) * P.N]) for c in range(n_chunks)])
    n_out = 2 * P.n_pack + 7
    W = _conv_like(rng, n_out, n_in, 144, 8)
    perm = rng.permutation(n_out)
    rows, Fo, packed = _run(F, P, chunks, W, perm, keys, engine)
    for c in range(n_chunks):
        want = R.extract(P, chunks[c])
        sel = rng.choice(P.N, 40, replace=False)
        assert np.array_equal(rows[c * P.N + sel], want[sel]), c
    sel = rng.choice(n_out, 30, replace=False)
    assert np.array_equal(Fo[sel], R.linear_rows(W[perm][sel], rows))
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(packed.shape[0]):
        assert np.array_equal(packed[g], R.pack(P, Fo[g * P.n_pack: (g + 1) * P.n_pack], keys)), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(packed[g])[pos[: seg.size]], seg), g


def test_native_pack_needs_keys_and_rejects_stale_handles():
    from paper_2509_01253_amd import fhelin as F
    import torch
    nt = F.fhelin_native_create(3, 4, 1, 3, 9, 3, 8)
    rows = torch.zeros((5, 2, 54), dtype=torch.int64, device="cuda")
    packed = torch.zeros((1, 2, 54), dtype=torch.int64, device="cuda")
    with pytest.raises(F.FhelinError) as e:
        F.fhelin_native_pack(nt, rows, packed)
    assert e.value.status == F.FHELIN_E_MISSING_GALOIS_KEY
    assert F.fhelin_native_pack_workspace(nt, 18) > 0
    F.fhelin_native_destroy(nt)
    with pytest.raises(F.FhelinError):
        F.fhelin_native_destroy(nt)


@pytest.mark.parametrize("t,alpha,gamma,beta,shape", [
    (3, 4, 1, 3, (3, 5, 4, 4, 3, 1)), (3, 4, 2, 3, (4, 6, 4, 4, 3, 2)), (5, 3, 1, 2, (6, 20, 4, 4, 1, 2)),
    (3, 7, 1, 6, (16, 16, 8, 8, 3, 1)), (3, 7, 2, 6, (64, 10, 1, 1, 1, 1)),
    # wider than 16 output channels: several channel groups, the last one padded
    (3, 4, 1, 3, (8, 40, 4, 4, 3, 1)), (5, 3, 2, 2, (4, 17, 3, 3, 3, 2)), (3, 7, 1, 6, (32, 64, 3, 3, 3, 1))])
def test_native_conv_layer_bit_exact(t, alpha, gamma, beta, shape):
    """The convolution kernel on extracted rows (channels-last windows, zero padding,
    strides 1 and 2, the FC case h = w = k = 1) with the shuffle as the output rows:
    element by element equal to the oracle's matrix product with the convolution's
    matrix, then packed, and decrypting to the integer layer."""
    import torch

    from paper_2509_01253_amd import fhelin as F
    c_in, c_out, h, w, k, st = shape
    print(f"native conv t={t} alpha={alpha} gamma={gamma} {shape}", flush=True)
    P = R.NativeParams(t, alpha, gamma, beta, 9, 3, 8, 2.0 ** 28)
    cl = R.NativeClient(P, 300 + t + alpha + gamma)
    keys = cl.keyset()
    rng = np.random.default_rng(310 + t + c_in)
    E = c_in * h * w
    n_chunks = (E + P.N - 1) // P.N
    x = rng.integers(0, 16, E)
    xs = np.zeros(n_chunks * P.N, np.int64)
    xs[:E] = x
    chunks = np.stack([cl.encrypt_powers(xs[c * P.N: (c + 1) * P.N]) for c in range(n_chunks)])
    wts = rng.integers(-8, 8, (c_out, c_in, k, k)).astype(np.int32)
    Wc = R.conv_matrix(c_in, c_out, h, w, k, st, wts)
    n_out = Wc.shape[0]
    out_row = rng.permutation(n_out).astype(np.int32)
    Wp = np.zeros_like(Wc)
    Wp[out_row] = Wc
    nt = F.fhelin_native_create(t, alpha, gamma, beta, 9, 3, 8, (t + alpha) % 2)
    try:
        F.fhelin_native_keys_load(nt, dev(np.stack([keys[d] for d in P.taus()])))
        rows = torch.zeros((n_chunks * P.N, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_extract(nt, dev(chunks), rows)
        out = torch.zeros((n_out, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_conv(nt, c_in, c_out, h, w, k, st, _i32(wts), _i32(out_row), rows, out)
        n_packs = (n_out + P.n_pack - 1) // P.n_pack
        packed = torch.zeros((n_packs, 2, P.N), dtype=torch.int64, device="cuda")
        F.fhelin_native_pack(nt, out, packed)
        got_rows, got, got_p = host(rows), host(out), host(packed)
    finally:
        F.fhelin_native_destroy(nt)
    sel = rng.choice(n_out, min(n_out, 40), replace=False)
    assert np.array_equal(got[sel], R.linear_rows(Wp[sel], got_rows[:E]))
    y = (Wp @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(n_packs):
        assert np.array_equal(got_p[g], R.pack(P, got[g * P.n_pack: (g + 1) * P.n_pack], keys)), g
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        assert np.array_equal(cl.decrypt(got_p[g])[pos[: seg.size]], seg), g
