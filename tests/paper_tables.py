"""Loader for the paper's operation-count tables (tests/golden/paper_tables.txt)."""
import os

_F = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_tables.txt")


def rows():
    out = []
    for line in open(_F):
        if line.startswith("#") or not line.strip():
            continue
        t, rel, ns, nP, nN, sp, nl, nL, nlist, ncontr, naive = line.split()
        out.append(dict(
            table=t, rel=bool(int(rel)), nsrc=int(ns), nP=int(nP), nN=int(nN),
            spins=None if sp == "all" else tuple(int(x) for x in sp.split(",")),
            n_lambda=int(nl), n_L=None if nL == "-" else int(nL),
            n_list=None if nlist == "-" else int(nlist),
            n_contr=None if ncontr == "-" else int(ncontr),
            naive=None if naive == "-" else float(naive)))
    return out


def row_id(r):
    sp = "all" if r["spins"] is None else "".join(map(str, r["spins"]))
    return f"{r['table']}-{r['nP']}{r['nN']}-{sp}"
