"""The cache-block model against the tiles' on-chip storage, per compiled shape
(the GPU side of the paper's model validation, Sec. III-B and IV-B).

For every compiled MWD tile shape (diamond width Dw, x lanes) of each stencil
and element type, the table gives:

  * C_S: the wavefront cache block of Eq. (3),
    N_xb [N_D Dw (Dw/2 - R + N_F) + 2R (Dw + W_w)], W_w = Dw - 2R + N_F, with one
    frontline (N_F = 1) and N_xb = lanes x element size (the x extent the tile
    holds, its recomputed ring included);
  * what the tile kernel holds on chip per workgroup: LDS bytes plus vector
    registers (registers per lane x 4 bytes x threads), the workgroups that fit
    one CU, and the register spill;
  * C_S and the held bytes as fractions of one CU's on-chip storage (160 KiB of
    LDS and a 512 KiB register file), against which the paper's rule of thumb
    (the model holds while the block fills at most about half the cache) is read;
  * the measured HBM traffic over the Eq. (5) model, from the model-validation
    summaries in profiles/ where one exists for the shape.

    python -m paper_1410_5561_amd.cacheblock [--out profiles/cache_block_table.txt]

Needs the GPU (kernel attributes come from the HIP runtime).
"""
from __future__ import annotations

import argparse
import glob
import os
import re

import paper_1410_5561_amd as S

ND = {"7c": 2, "7v": 9, "25c": 2, "25v": 15}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}
CU_ONCHIP = (160 + 512) * 1024
PKG = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(os.path.dirname(PKG), "profiles")


def cache_block(kind: str, elem: int, dw: int, lanes: int, nf: int = 1) -> float:
    """Eq. (3) in bytes."""
    R, nd = RADIUS[kind], ND[kind]
    nxb = lanes * elem
    ww = dw - 2 * R + nf
    return nxb * (nd * dw * (dw / 2 - R + nf) + 2 * R * (dw + ww))


def measured_ratios() -> dict:
    """{(kind, dtype, 'DWxLANES'): traffic / model} from the model-validation summaries."""
    out = {}
    for path in glob.glob(os.path.join(PROFILES, "model_validation_*.txt")):
        with open(path) as f:
            text = f.read()
        m = re.search(r"workload \S+ \((\w+) (f\d\d)\)", text)
        if not m:
            continue
        kind, dtype = m.group(1), m.group(2)
        for line in text.splitlines():
            cols = line.split()
            if len(cols) >= 5 and re.fullmatch(r"\d+x\d+", cols[0]):
                try:
                    out[(kind, dtype, cols[0])] = float(cols[4])
                except ValueError:
                    pass
    return out


def table() -> list[str]:
    ratios = measured_ratios()
    lines = [
        "# Eq. (3) cache block (N_F = 1, N_xb = lanes x element size) against what each compiled",
        "# MWD tile kernel holds on chip, and the measured HBM traffic over the Eq. (5) model.",
        "# CU on-chip storage: 160 KiB LDS + 512 KiB vector registers = 672 KiB.",
        "# command: python -m paper_1410_5561_amd.cacheblock",
        "%-4s %-4s %-7s %9s %6s %9s %9s %9s %6s %7s %7s %6s" % (
            "kind", "type", "shape", "C_S KiB", "C_S/CU", "LDS KiB", "VGPR KiB", "held KiB", "WG/CU",
            "held/CU", "spill B", "t/m"),
    ]
    for kind in ("7c", "7v", "25c", "25v"):
        for dtype, elem in (("f64", 8), ("f32", 4)):
            for dw in (4, 8, 10, 16):
                for lanes in (64, 128, 256):
                    try:
                        r = S.stencil_kernel_resources(kind, dtype, dw, lanes)
                    except S.StencilError:
                        continue
                    cs = cache_block(kind, elem, dw, lanes)
                    vgpr_b = r["vgprs"] * 4 * r["threads"]
                    held = r["lds_bytes"] + vgpr_b
                    ratio = ratios.get((kind, dtype, "%dx%d" % (dw, lanes)))
                    lines.append("%-4s %-4s %-7s %9.1f %6.2f %9.1f %9.1f %9.1f %6d %7.2f %7d %6s" % (
                        kind, dtype, "%dx%d" % (dw, lanes), cs / 1024, cs / CU_ONCHIP, r["lds_bytes"] / 1024,
                        vgpr_b / 1024, held / 1024, r["workgroups_per_cu"],
                        held * max(1, r["workgroups_per_cu"]) / CU_ONCHIP, r["scratch_bytes_per_lane"],
                        "%.3f" % ratio if ratio else "-"))
    return lines


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    lines = table()
    text = "\n".join(lines) + "\n"
    print(text, end="")
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            f.write(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
