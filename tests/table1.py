"""Loader for tests/golden/table1.tsv (Table 1 of the paper, as printed)."""
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1.tsv")


def rows():
    out = []
    with open(PATH) as f:
        lines = [ln.rstrip("\n") for ln in f if not ln.startswith("#")]
    header = lines[0].split("\t")
    for ln in lines[1:]:
        rec = dict(zip(header, ln.split("\t")))
        out.append({"L": int(rec["L"]), "F": rec["F"], "dagger": rec["dagger"] == "1",
                    "hex": rec["hex"], "PSL": int(rec["PSL"])})
    return out
