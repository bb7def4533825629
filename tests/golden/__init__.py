"""Readers for the small text fixtures in this folder (each cites its source)."""
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def worked_example() -> dict:
    """Parsed worked_example.txt (Section 2.2 of the paper)."""
    out = {}
    with open(os.path.join(_HERE, "worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, _, rest = line.partition(":")
            out[name.strip()] = rest.split()
    ex = {
        "keys": [k.encode() for k in out["keys"]],
        "sorted": [k.encode() for k in out["sorted"]],
        "counts": {int(a, 16): int(b) for a, b in (t.split(":") for t in out["first_byte_counts"])},
        "offsets": {int(a, 16): int(b) for a, b in (t.split(":") for t in out["first_byte_offsets"])},
        "c_second": [int(t, 16) for t in out["bucket_63_second_bytes"]],
    }
    return ex


def pad_key(k: bytes) -> bytes:
    return k + b"\x00" * (10 - len(k))
