"""Limits the host runtime relies on, checked from the headers (no GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_08371_amd", "csrc")


def _header_int(path, pattern):
    with open(path) as f:
        return [int(v) for v in re.search(pattern, f.read(), re.S).groups()]


def test_partial_sum_block_of_a_macro_fits_32_bit_offsets():
    """The seam gather addresses one macro's partial sums by 32-bit byte offsets;
    at the largest P2 level every tile shape keeps that block below 4 GiB
    (vector fields, FP64), so the host guard that refuses larger blocks never
    fires for a supported operator."""
    (lmax,) = _header_int(os.path.join(ROOT, "include", "tetmf.h"), r"#define TMF_MAX_LEVEL_P2 (\d+)")
    with open(os.path.join(CSRC, "tmf_internal.h")) as f:
        cfg = re.search(r"kTileCfg\[kNumTileCfg\]\[3\] = \{(.*?)\};", f.read(), re.S).group(1)
    shapes = [tuple(int(v) for v in t.split(",")) for t in re.findall(r"\{([^{}]*)\}", cfg)]
    assert len(shapes) >= 1
    n = 2 ** lmax
    for TX, TY, TZ in shapes:
        tiles = sum(1 for bz in range(0, n, TZ) for by in range(0, n - bz, TY) for bx in range(0, n - bz - by, TX))
        R = (2 * TX + 1) * (2 * TY + 1) * (2 * TZ + 1)
        assert tiles * R * 3 * 8 < 2 ** 32, (TX, TY, TZ)
