"""The ResNet-18 layer list as the server sees it (CPU): 21 rounds (stem, 16
block convs, 3 downsampling 1x1 convs, FC 512->200), their key-switch and
multiply-accumulate counts for the N=2^16 multiplexed packing, and the
plaintext forward pass (client work between rounds) against a direct
implementation."""
import numpy as np

from oracle import oracle as O
from paper_2509_01253_amd import resnet, synth


def test_layer_list_and_counts():
    specs = resnet18_layers = resnet.resnet18_layers()
    assert len(specs) == 21
    assert sum(1 for s in specs if s.kind == "conv" and s.k == 3) == 17
    assert sum(1 for s in specs if s.kind == "conv" and s.k == 1) == 3
    assert specs[-1].kind == "fc" and specs[-1].c_in == 512 and specs[-1].c_out == 200 and specs[-1].fc_n == 512
    S = 1 << 15
    ks, macs = [], 0
    for s in specs:
        if s.kind == "conv":
            cs = O.ConvShape(s.c_in, s.c_out, s.h, s.w, s.k)
            sc = O.conv_schedule(cs, S)
        else:
            sc = O.fc_schedule(s.fc_n, 16)
        ks.append(sc.n_in * sum(1 for r in sc.rb if r) + sc.n_out * sum(1 for r in sc.gk if r))
        macs += sc.n_out * sc.n_in * sc.G * sc.B
    # stem 64; stage-1 convs 120 each; the rest follow from the channel blocking
    assert ks[0] == 64 and ks[1:5] == [120] * 4
    assert sum(ks) == 5273 - 46 + ks[-1]
    assert macs - 512 == 91712 - 512


def test_forward_matches_direct_resnet():
    st = synth.Stream(77)
    specs = resnet.resnet18_layers(h=8, w=8, widths=(4, 8, 8, 16), n_classes=10)
    W = resnet.init_weights(specs, st)
    fw = resnet.Forward(specs, W)
    x = st.uniform(3 * 64, 0, 1).reshape(3, 8, 8)
    got = fw.run(x, fw.plain_linear)

    def conv_s(Wc, a, stride):
        return resnet.conv_same(Wc, a)[:, ::stride, ::stride]

    relu = lambda a: np.maximum(a, 0)
    h = relu(conv_s(W["stem"], x, 1))
    for s, c in enumerate((4, 8, 8, 16)):
        for b in range(2):
            stride = 2 if s > 0 and b == 0 else 1
            pre = f"s{s + 1}b{b + 1}"
            a = relu(conv_s(W[pre + "c1"], h, stride))
            y = conv_s(W[pre + "c2"], a, 1)
            sc = conv_s(W[pre + "ds"], h, 2) if stride == 2 and (pre + "ds") in W else h
            h = relu(y + sc)
    want = W["fc"] @ h.mean(axis=(1, 2))
    assert np.allclose(got, want)


def test_shuffled_rounds_give_the_same_logits():
    """With every layer's seeded shuffle and the previous round's unshuffle folded
    into its weights (W'[t][u] = W[perm_out[t]][perm_in[u]], the oracle's folding),
    the client works on shuffled activations only -- ReLU, residual additions,
    subsampling and pooling in shuffled order -- and still receives the network's
    logits; intermediate activations are the true ones permuted (the client sees no
    channel order), and every layer but the FC shuffles its output."""
    st = synth.Stream(78)
    specs = resnet.resnet18_layers(h=8, w=8, widths=(4, 8, 8, 16), n_classes=10)
    W = resnet.init_weights(specs, st.sub(synth.TAG_W))
    perms = resnet.shuffle_perms(specs, st.sub(synth.TAG_PERM))
    assert set(perms) == {s.name for s in specs}
    assert perms["stem"][1] is None and perms["fc"][0] is None
    for s in specs[:-1]:
        assert sorted(perms[s.name][0]) == list(range(s.c_out))
    fw = resnet.Forward(specs, W)
    x = st.uniform(3 * 64, 0, 1).reshape(3, 8, 8)
    seen = {}

    def shuffled(spec, a):
        po, pi = perms[spec.name]
        Wp = O.fold_permutations(W[spec.name], po, pi)
        out = O.conv_ref(Wp, a) if spec.kind == "conv" else Wp @ a
        seen[spec.name] = out
        return out

    def plain(spec, a):
        out = O.conv_ref(W[spec.name], a) if spec.kind == "conv" else W[spec.name] @ a
        seen["plain_" + spec.name] = out
        return out

    got = fw.run(x, shuffled)
    want = fw.run(x, plain)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the stem's output reaches the client permuted, not in the true order
    p = perms["stem"][0]
    assert np.allclose(seen["stem"], seen["plain_stem"][p])
    assert not np.allclose(seen["stem"], seen["plain_stem"])
