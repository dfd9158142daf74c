"""Write tests/golden/instances.json: the structure of the standard seeded
code instances as computed by the oracle (and only the oracle)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from lead_inputs import standard, STANDARD  # noqa: E402
from oracle.oracle import OracleCode  # noqa: E402


def main():
    out = {}
    for name in STANDARD:
        spec = standard(name)
        info = OracleCode.from_spec(spec).info
        out[name] = dict(spec=spec.describe(), n=info.n, r=list(info.r), m=list(info.m),
                         rank=list(info.rank), k=info.k, eloc=list(info.eloc))
    with open(os.path.join(HERE, "instances.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
