"""Error gates of the GPU parity tests (rel_mag, see the parity test module).

The target is 1e-12 for the FP64 path and 1e-6 for the mixed paths that claim
it (FP32, split-bf16x6, scaled FP16x3). Split-bf16x3 does not claim it: two
bf16 terms hold 16 significant bits, and where a few rank terms dominate a
value its error reaches about 2^-17 of it (2.3e-6 measured on a small box).
It is checked against the bound its arithmetic guarantees instead:
per product x y, with x = x0 + x1 + ex, both terms rounded to nearest,
|x1| <= 2^-8 (1 + 2^-8) |x| and |ex| <= 2^-16 |x|, the three kept products
miss x1 y1 + (x0 + x1) ey + ex (y0 + y1) + ex ey, at most
3 * 2^-16 * (1 + 2^-7) |x y|; rounding the two operands to FP32 adds
2 * 2^-24 and the FP32 sum of 3K products (K rank terms) at most 3K * 2^-24,
all relative to sum_r |terms| = the same potential with |Z| (rel_mag).
"""

GATES = {"f64": 1e-12, "f32": 1e-6, "bf16x6": 1e-6, "f16x3": 1e-6}


def bf16x3_bound(K):
    return 3 * 2.0 ** -16 * (1 + 2.0 ** -7) + (3 * K + 2) * 2.0 ** -24


def gate(precision, K):
    """rel_mag gate of a reconstruction with K rank terms."""
    return bf16x3_bound(K) if precision == "bf16x3" else GATES[precision]
