"""Write the radix-split tuning table of this GPU.

Usage: python -m paper_2410_15880_amd.autotune [lg_lo lg_hi [out_path]]

Times the device search for every split candidate per size class (halves of
2^lg keys) and writes paper_2410_15880_amd/tuning/mi355x.txt, which contexts
load at creation.
"""
import sys

import paper_2410_15880_amd as R


def main():
    lo = int(sys.argv[1]) if len(sys.argv) > 1 else 12
    hi = int(sys.argv[2]) if len(sys.argv) > 2 else 27
    out = sys.argv[3] if len(sys.argv) > 3 else R.TUNING_PATH
    with R.Context(0) as ctx:
        ctx.autotune(lo, hi, out)
    print(open(out).read(), end="", flush=True)


if __name__ == "__main__":
    main()
