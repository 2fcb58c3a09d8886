"""A ResNet-18-shaped stack of encrypted linear layers (reduced widths and
resolution so the test stays small; same structure: stem, four stages with
strided and downsampling convs, FC): one captured graph per layer, replayed
for two inferences; client decrypt / ReLU / residual / re-encrypt between
rounds.  Every layer folds its seeded channel shuffle and the previous round's
unshuffle into its weights, so the client only ever holds shuffled activations;
the decrypted logits still match the FP64 network, and one layer's output
ciphertext is checked bit-for-bit against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import resnet, synth
from tests.gpu_util import dev, host, keys_at
from tests.helpers import Client, encode_pts

pytestmark = pytest.mark.gpu


class GpuClient:
    def __init__(self, prm, seed):
        self.prm = prm
        self.cl = Client(prm, seed)

    def encrypt(self, slots, level):
        return dev(np.stack([self.cl.encrypt_slots(z, level, self.prm.scale) for z in slots]))

    def decrypt(self, y, level, scale):
        got = host(y)
        return np.stack([self.cl.decrypt_slots(got[i, :, :level], level, scale).real for i in range(got.shape[0])])

    def keys(self, galois, level):
        ks = O.KeySet(list(galois), np.stack([self.cl.galois_key(g) for g in galois]))
        return dev(keys_at(self.prm, ks, level))


def test_resnet_stack_graphs():
    import torch

    from paper_2509_01253_amd import fhelin as F
    print("resnet stack", flush=True)
    prm = O.make_params(12, 3, 2, 3, 50, 2.0 ** 40)
    level = 3
    st = synth.Stream(synth.master_seed(4))
    specs = resnet.resnet18_layers(h=16, w=16, widths=(8, 16, 32, 64), n_classes=10)
    W = resnet.init_weights(specs, st.sub(synth.TAG_W))
    client = GpuClient(prm, synth.master_seed(4))
    ctx = F.fhelin_ctx_create(prm.log_n, prm.q, prm.p, prm.dnum)
    stream = torch.cuda.Stream()
    flags = F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN
    perms = resnet.shuffle_perms(specs, st.sub(synth.TAG_PERM))
    stack = resnet.EncryptedStack(F, ctx, prm.log_n, specs, W, client, level, prm.scale, prm.q[level - 1], flags,
                                  stream, perms=perms)

    def plain(spec, a):  # the FP64 layer, unshuffled: the oracle's convolution / matrix product
        return O.conv_ref(W[spec.name], a) if spec.kind == "conv" else W[spec.name] @ a

    try:
        fw = resnet.Forward(specs, W)
        for img in range(2):
            x = st.sub(synth.TAG_X).sub(img).uniform(3 * 256, 0, 1).reshape(3, 16, 16)
            want = fw.run(x, plain)
            got = fw.run(x, stack.linear)
            err = np.abs(got - want).max() / np.abs(want).max()
            print(f"image {img}: logits rel err {err:.2e}", flush=True)
            assert err < 1e-3
        # one layer of the stack (its plan and keys) bit-exact against the oracle, from
        # oracle-encoded plaintexts and a fresh encryption
        sp = stack.layers["s2b1c2"]["spec"]
        L = stack.layers[sp.name]
        cs = O.ConvShape(sp.c_in, sp.c_out, sp.h, sp.w, sp.k)
        sched = O.conv_schedule(cs, prm.S)
        pts = encode_pts(prm, O.conv_slots(W[sp.name], cs, prm.S), level, prm.scale)
        pset = F.fhelin_pt_import(ctx, dev(pts.reshape(-1, level + prm.K, prm.N)), level=level)
        xs = stack.pack(sp, st.uniform(sp.c_in * sp.h * sp.w, 0, 1).reshape(sp.c_in, sp.h, sp.w))
        cts = np.stack([client.cl.encrypt_slots(z, level, prm.scale) for z in xs])
        y = dev(np.zeros((sched.n_out, 2, level, prm.N), np.uint64))
        F.fhelin_linear_apply(ctx, L["plan"], L["ks"], pset, dev(cts), [level] * len(cts), y,
                              [level - 1] * sched.n_out, flags)
        gal = F.fhelin_plan_galois(L["plan"])
        keys = O.KeySet(gal, np.stack([client.cl.galois_key(g) for g in gal]))
        want = O.linear(prm, cts, level, sched, pts, keys, hoist_moddown=True)
        yout = host(y)
        for o in range(sched.n_out):
            assert np.array_equal(yout[o, :, : level - 1], O.rescale(prm, want[o], level)), o
        F.fhelin_ptset_release(pset)
    finally:
        stack.close()
        F.fhelin_ctx_destroy(ctx)
