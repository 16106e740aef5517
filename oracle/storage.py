"""What the reduced-precision storage classes of the GPU path represent.

These are additions to the paper (which computes in double precision): the
solver keeps its iterated vectors in FP32, or in FP16 with one FP32 scale per
site, and its links in FP32 or FP16 with the third row rebuilt.  The oracle
defines the rounded values such storage holds, so that a reduced-precision
operator can be compared with the exact operator applied to the same rounded
inputs.

* F32 spinor: each complex component rounded to complex64.
* F16S spinor: the 24 reals of a site are first rounded to FP32; the site's
  scale is the largest of their magnitudes (FP32); each real is stored as the
  FP16 nearest to (value / scale) computed in FP32; a site of zeros has scale
  0 and stores zeros.  The represented value is FP32(half) * scale.
* Reconstruct-12 links: rows 0 and 1 of each SU(3) link are stored rounded
  (each real rounded once, from FP64 straight to the nearest FP32 or FP16, ties
  to even; no intermediate FP32 step for FP16); row 2 is conj(row0 x row1),
  exact for a special unitary matrix.

Pins: tests/test_oracle_storage.py, tests/test_half_rounding.py (FP16 rounding
against an exhaustive nearest-value search on doubles where rounding through
FP32 first would differ).
"""
import numpy as np


def round_f32(psi):
    return psi.astype(np.complex64).astype(np.complex128)


def f16s_quantize(psi):
    """psi [...site..., 3, 4] complex128 -> (halves [..., 24] float16, scale [...] float32).
    Reals are ordered (colour, spin, re/im) with re/im fastest."""
    v = psi.astype(np.complex64)
    re = np.stack([v.real, v.imag], axis=-1).reshape(psi.shape[:-2] + (24,)).astype(np.float32)
    scale = np.abs(re).max(axis=-1).astype(np.float32)
    safe = np.where(scale > 0, scale, np.float32(1.0)).astype(np.float32)
    q = (re / safe[..., None]).astype(np.float32).astype(np.float16)
    q = np.where(scale[..., None] > 0, q, np.float16(0))
    return q, scale


def f16s_dequantize(q, scale):
    re = q.astype(np.float32) * scale[..., None].astype(np.float32)
    re = re.reshape(q.shape[:-1] + (3, 4, 2)).astype(np.float64)
    return re[..., 0] + 1j * re[..., 1]


def round_f16s(psi):
    return f16s_dequantize(*f16s_quantize(psi))


def reconstruct12(rows01):
    """rows01 [..., 2, 3] -> full [..., 3, 3] with row2 = conj(row0 x row1)."""
    a, b = rows01[..., 0, :], rows01[..., 1, :]
    c = np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                  a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                  a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)
    return np.concatenate([rows01, np.conj(c)[..., None, :]], axis=-2)


def round_links_r12(U, dtype):
    """Links as a reconstruct-12 store in ``dtype`` (np.complex64 or 'f16') represents them."""
    rows = U[..., 0:2, :]
    if dtype == "f16":
        re = rows.real.astype(np.float16).astype(np.float64)
        im = rows.imag.astype(np.float16).astype(np.float64)
        rows = re + 1j * im
    else:
        rows = rows.astype(np.complex64).astype(np.complex128)
    return reconstruct12(rows)
