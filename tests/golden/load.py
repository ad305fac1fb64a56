"""Parsers for the hand-worked fixtures in this folder."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def sdtw_cases():
    recs, cur = [], {}
    with open(os.path.join(HERE, "sdtw_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if line.startswith("#"):
                continue
            if not line:
                if cur:
                    recs.append(cur)
                    cur = {}
                continue
            key, _, val = line.partition(":")
            val = val.strip()
            if key in ("NAME", "CITE"):
                cur[key] = val
            elif key.startswith("ROW"):
                cur.setdefault("ROWS", []).append([int(v) for v in val.split()])
            elif key in ("X", "Y"):
                cur[key] = [int(v) for v in val.split()]
            else:
                cur[key] = int(val)
    if cur:
        recs.append(cur)
    return recs


def prep_cases():
    out = {}
    with open(os.path.join(HERE, "prep_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(":")
            out[key] = [float(v) for v in val.split()]
    return out
