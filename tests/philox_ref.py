"""Host reference of the training-vector generator: Philox4x32-10 (Salmon,
Moraes, Dror & Shaw, SC'11) written from its published definition, and the
Box-Muller transform.  Independent of the GPU code; pinned by the published
known-answer vectors in test_gpu_nn.py / test_philox_ref.py."""
import numpy as np

M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c = [int(v) & MASK for v in ctr]
    k = [int(v) & MASK for v in key]
    for _ in range(10):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & MASK, p1 & MASK, ((p0 >> 32) ^ c[3] ^ k[1]) & MASK, p0 & MASK]
        k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
    return c


def site_normals(lex, seed, step):
    """The 24 reals (colour-major, spin, re/im) of canonical site lex."""
    key = (seed & MASK, (seed >> 32) & MASK)
    out = []
    for b in range(6):
        w = philox4x32_10((lex, b, step & MASK, (step >> 32) & MASK), key)
        for h in range(2):
            u0 = (w[2 * h] + 0.5) * 2.0 ** -32
            u1 = (w[2 * h + 1] + 0.5) * 2.0 ** -32
            r = np.sqrt(-2.0 * np.log(u0))
            out += [r * np.cos(2 * np.pi * u1), r * np.sin(2 * np.pi * u1)]
    return np.array(out)
