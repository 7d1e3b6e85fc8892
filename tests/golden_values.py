"""Reader for the closed-form fixtures in tests/golden/closed_forms.txt."""

import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.txt")


def closed_forms():
    out = {}
    with open(_PATH) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                out[k.strip()] = float(v)
    return out
