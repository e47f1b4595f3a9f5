"""Shared helpers of the GPU parity tests (no method arithmetic)."""
import numpy as np

GROUPS = {"rho": slice(0, 1), "j": slice(1, 4), "P": slice(4, 10)}
# quantization steps of the codec variables rho, u, N (Sec. 5.3 ranges / 65535)
DELTA = np.array([0.7 / 65535] + [0.8 / 65535] * 3 + [0.2 / 65535] * 6)
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def group_rel_err(got, ref):
    """Per moment group: max |got - ref| / max |ref|."""
    out = {}
    for name, g in GROUPS.items():
        den = max(np.abs(ref[g]).max(), 1e-30)
        out[name] = float(np.abs(np.asarray(got[g], dtype=np.float64) - ref[g]).max() / den)
    return out


def codec_vars(m):
    """(rho, u, N = P - rho u u) of a moment field, shape (10, ...)."""
    m = np.asarray(m, dtype=np.float64)
    rho = m[0]
    u = m[1:4] / rho
    N = [m[4 + p] - rho * u[a] * u[b] for p, (a, b) in enumerate(PAIRS)]
    return np.stack([rho, *u, *N])


def unpack(w):
    w = np.asarray(w, dtype=np.uint32)
    q = np.empty((10,) + w.shape[1:], dtype=np.int64)
    q[0::2] = w & 0xFFFF
    q[1::2] = w >> 16
    return q


def fluid(mask, shape):
    return np.ones(shape[1:], bool) if mask is None else (mask == 0)


def unpack_packed(w, b1, b2):
    """Codes of the b1 / b2 packed layout (rho, ux, uy, uz with b1 bits, N
    with b2 bits, concatenated low bit first across a cell's words)."""
    w = np.asarray(w, dtype=np.uint64)
    out = np.empty((10,) + w.shape[1:], dtype=np.int64)
    o = 0
    for k in range(10):
        b = b1 if k < 4 else b2
        i, s = divmod(o, 32)
        v = w[i] >> np.uint64(s)
        if s + b > 32:
            v = v | (w[i + 1] << np.uint64(32 - s))
        out[k] = (v & np.uint64((1 << b) - 1)).astype(np.int64)
        o += b
    return out


def delta_bits(b1, b2):
    """Quantization steps of (rho, u, N) with b1 / b2 bits."""
    return np.array([0.7 / (2 ** b1 - 1)] + [0.8 / (2 ** b1 - 1)] * 3 + [0.2 / (2 ** b2 - 1)] * 6)
