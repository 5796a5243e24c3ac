"""Host model (numpy) of the 16-bit offset population words of the
LBM_STORAGE_F16_OFS / LBM_STORAGE_BF16_OFS formats, written from the format's
description in the public header.  Test infrastructure: used to build device
states, to read them back and to bound the rounding the format introduces.

Word layout per site (10 words of 32 bits):
  word 0, 1 : R_0, B_0 as float;
  word 1 + i: link i = 1..8, low half = 1024 (f_i - fref_i) / fref_i in FP16
              or BF16, high half = stored colour s_i / (4 fref_i) in FP16
              (clamped to magnitude below 2), bit 14 set if s_i is the blue
              population; s_i is the colour of smaller magnitude, the other
              colour is f_i - s_i.
All arithmetic is FP32, as on the device.
"""
import numpy as np

CLS = [0, 2, 1, 2, 1, 2, 1, 2, 1]   # link class: rest, diagonal (odd), axis (even)
ZMAX = np.float32(1.9990234375)      # largest FP16 value below 2 (bit 14 clear)
LINK_OF_WORD = [0, 0] + list(range(1, 9))


def frefs(params):
    """fref per link class and its FP32 reciprocal: (9/5) w rho0_R (1 - alpha_R)."""
    moving = float(params["rho0_R"]) * (1.0 - float(params["alpha_R"]))
    fr = np.array([1.0, 0.2 * moving, 0.05 * moving], dtype=np.float32)
    inv = (1.0 / fr.astype(np.float64)).astype(np.float32)
    return fr, inv


def offset_quanta(params):
    """fref / 1024 and 1024 / fref in FP32."""
    fr, _ = frefs(params)
    f = fr.astype(np.float64)
    return (f / 1024.0).astype(np.float32), (1024.0 / f).astype(np.float32)


def colour_units(params):
    """4 fref and 1 / (4 fref) in FP32."""
    fr, _ = frefs(params)
    f = fr.astype(np.float64)
    return (4.0 * f).astype(np.float32), (0.25 / f).astype(np.float32)


def f16_bits(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).view(np.uint16).astype(np.uint32)


def f16_value(h):
    return np.asarray(h, dtype=np.uint32).astype(np.uint16).view(np.float16).astype(np.float32)


def bf16_bits(x):
    """Round-to-nearest-even FP32 -> BF16 (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint32) & 0xFFFF


def bf16_value(h):
    return (np.asarray(h, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32)


LOW = {"f16": (f16_bits, f16_value), "bf16": (bf16_bits, bf16_value)}


def encode(R, B, params, fmt):
    """[9, ...] red and blue populations -> [10, ...] uint32 words."""
    enc_low, _ = LOW[fmt]
    R = np.asarray(R, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    fr, _ = frefs(params)
    _, inv_q = offset_quanta(params)
    _, inv_sq = colour_units(params)
    w = np.empty((10,) + R.shape[1:], dtype=np.uint32)
    w[0] = R[0].view(np.uint32)
    w[1] = B[0].view(np.uint32)
    for i in range(1, 9):
        k = CLS[i]
        f = R[i] + B[i]
        blue = np.abs(B[i]) < np.abs(R[i])
        s = np.where(blue, B[i], R[i])
        z = np.clip((s * inv_sq[k]).astype(np.float32), -ZMAX, ZMAX).astype(np.float32)
        hc = f16_bits(z) | np.where(blue, 0x4000, 0).astype(np.uint32)
        w[1 + i] = enc_low(((f - fr[k]).astype(np.float32) * inv_q[k]).astype(np.float32)) | (hc << 16)
    return w


def decode(w, params, fmt):
    """[10, ...] words -> (R, B) [9, ...] float32."""
    _, dec_low = LOW[fmt]
    w = np.asarray(w).view(np.uint32) if np.asarray(w).dtype != np.uint32 else np.asarray(w)
    fr, _ = frefs(params)
    q, _ = offset_quanta(params)
    sq, _ = colour_units(params)
    R = np.empty((9,) + w.shape[1:], dtype=np.float32)
    B = np.empty_like(R)
    R[0] = w[0].view(np.float32)
    B[0] = w[1].view(np.float32)
    for i in range(1, 9):
        k = CLS[i]
        v = w[1 + i]
        # f = fma(low, fref / 1024, fref): the product of an FP16 or BF16 value
        # and an FP32 value is exact in FP64, the sum is rounded once to FP32
        f = (np.float64(fr[k]) + dec_low(v & 0xFFFF).astype(np.float64) * np.float64(q[k])).astype(np.float32)
        hc = v >> 16
        s = (f16_value(hc & 0xBFFF) * sq[k]).astype(np.float32)
        o = (f - s).astype(np.float32)
        blue = (hc & 0x4000) != 0
        R[i] = np.where(blue, o, s)
        B[i] = np.where(blue, s, o)
    return R, B


def decode_pair(w, params, fmt):
    R, B = decode(w, params, fmt)
    return np.stack([R, B]).astype(np.float64)


def rounding_bound(ref, params, fmt):
    """Per-element bound [2, 9, ...] of |decode(encode(x)) - x| for x near
    ref: one unit in the last place of the stored offset and of the stored
    colour (relative 2^-10 of FP16 values, 2^-7 of BF16 values, plus FP16's
    subnormal spacing), and the FP32 arithmetic of the two conversions;
    FP32 words (rest link) are exact."""
    ref = np.asarray(ref, dtype=np.float64)
    fr, _ = frefs(params)
    e_low = 2.0 ** -10 if fmt == "f16" else 2.0 ** -7
    tol = np.empty_like(ref)
    tol[:, 0] = 0.0
    for i in range(1, 9):
        f = ref[0, i] + ref[1, i]
        s = np.minimum(np.abs(ref[0, i]), np.abs(ref[1, i]))
        t = (e_low * np.abs(f - fr[CLS[i]]) + 2.0 ** -34 * fr[CLS[i]]      # offset: ulp, subnormal spacing
             + 2.0 ** -10 * s + 2.0 ** -22 * fr[CLS[i]]                    # stored colour (unit 4 fref)
             + 2.0 ** -22 * (np.abs(f) + s))                               # FP32 arithmetic
        tol[0, i] = t
        tol[1, i] = t
    return tol


def pull_words(W, walls):
    """One streaming step of a pull-layout word buffer W [10, ny, nx] on the
    host: word q of link i at r comes from r - c_i, or from the reversed
    link's word at r when r - c_i is a solid row.  Returns the full lattice
    with the solid rows unchanged."""
    from oracle.lattice import C, OPP
    W = np.asarray(W)
    ny = W.shape[1]
    out = W.copy()
    for q in range(10):
        i = LINK_OF_WORD[q]
        cx, cy = C[i]
        g = np.roll(np.roll(W[q], cx, axis=-1), cy, axis=-2)
        if walls:
            bq = q if q < 2 else 1 + OPP[i]
            if cy == 1:
                g[1] = W[bq, 1]
            elif cy == -1:
                g[ny - 2] = W[bq, ny - 2]
            out[q, 1:ny - 1] = g[1:ny - 1]
        else:
            out[q] = g
    return out
