"""Write the stored expected values under tests/golden/ from the CPU oracle.

Only the oracle is called.  The values are not printed in the paper (it prints
no random numbers); they anchor the oracle against accidental change and give
the GPU tests fixed vectors.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def hexs(v):
    return format(v, "x")


def main():
    lux = [24, 218, 404, 794, 2048]
    doc = {
        "about": "RANLUX++ oracle vectors: m = 2^576 - 2^240 + 1, a = b^-1 mod m, "
                 "A_p = a^p mod m, seed(id) = A_p^(2^96 id), 48-bit fields oldest pair first",
        "multipliers": {str(p): hexs(O.multiplier(p)) for p in lux},
        "seed_multipliers": {str(p): hexs(O.seed_multiplier(p)) for p in lux},
        "streams": [],
        "skips": [],
    }
    for p in lux:
        for sid in (0, 1, 2, 65535, 2 ** 40 + 3):
            x0 = O.seed(sid, p)
            vals, x1, pos1 = O.draws(x0, 0, p, 40)
            doc["streams"].append({"p": p, "id": sid, "seed_x": hexs(x0),
                                   "first40": [hexs(v) for v in vals],
                                   "x_after40": hexs(x1), "pos_after40": pos1})
    for k in (0, 1, 2, 15, 16, 255, 256, 2 ** 32 + 1, 2 ** 63 + 12345, 2 ** 64 - 1):
        x0 = O.seed(5, 2048)
        doc["skips"].append({"p": 2048, "id": 5, "k": str(k), "x": hexs(O.skip(x0, k, 2048))})
    with open(os.path.join(HERE, "oracle_vectors.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
