"""Readings study -- TEST INFRASTRUCTURE ONLY (calls nothing but the oracle).

The paper's code-capacity tables (unrotated surface code, depolarizing
noise, T = 25: the Appendix figures "fraction of calls to MWPM" and "Code
capacity performance of our algorithms", stored with their citation in
tests/golden/paper_code_capacity_unrotated.txt) are recomputed with the FP64
oracle under several readings of what the paper leaves open:

  z       the Z-error decoding graph only (the reading the library uses for
          its reported logical error rates): a shot fails if the Z part fails,
          never converges if the Z part never converges;
  xz      both error types, each decoded on its own graph from the same
          depolarizing draw: a shot fails if either part fails and calls the
          fallback if either part never converges;
  xz-lit  as xz with the update indices of Sec. II.B taken literally, which
          repeats every flooding iteration, so T = 25 literal iterations are
          13 flooding ones;
  xz-blk  as xz with the block-maxima forced convergence of Sec. II.D,
          conflicts matched to the boundary (BP4MF only);
  xz-xor  as xz with a candidate's weight taken as that of the XOR of its
          matched paths (BP4MF only).

The X part is decoded on the same graph through the code's transposition
symmetry: the qubit at (r, c) of the (2d-1) x (2d-1) layout maps to (c, r),
Z checks to X checks, and the Z logical on data column 0 to the X logical on
data row 0, so an X error is a Z error of the transposed code with the same
syndrome (checked below on every qubit) and observable.

    python oracle/readings.py [--quick] [--threads N]

prints markdown tables of the oracle's values next to the paper's;
--threshold SHOTS instead prints the xz logical error rates of BP4M and BP4MF
over the threshold region (d = 5, 9, 13; p = 0.10 .. 0.15); --bbp4mf SHOTS
those of B-BP4MF (z and xz) next to the paper's printed code-capacity panel
(tests/golden/paper_bbp4mf_code_capacity_unrotated.txt).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_code_capacity_unrotated.txt")
DEPOL_TAG = 0x44455031          # fourth counter word of the depolarizing draw


def paper_tables():
    t = {}
    for ln in open(GOLDEN):
        if ln.startswith("#") or not ln.strip():
            continue
        name, d, p, v = ln.split()
        t[(name, int(d), round(float(p), 2))] = float(v)
    return t


def qubit_index(d, r, c):
    """Index of the data qubit at (r, c), (r + c) even, rows numbered top
    down with d qubits on even rows and d - 1 on odd rows."""
    before = sum(d if rr % 2 == 0 else d - 1 for rr in range(r))
    return before + c // 2


def transposition(d, T, with_xmap=False):
    """Qubit permutation (r, c) -> (c, r) and the map from Z-check index to
    the X-check index of the transposed position; checked against the Tanner
    graph: every qubit's Z checks become its image's X checks.  With
    with_xmap, also the map from X-check index to the Z-check index of the
    transposed position, checked the same way."""
    n = 2 * d - 1
    perm = np.zeros(T.n_q, dtype=np.int64)
    col0 = []
    for r in range(n):
        for c in range(n):
            if (r + c) % 2:
                continue
            v = qubit_index(d, r, c)
            perm[v] = qubit_index(d, c, r)
            if c == 0:
                col0.append(v)
    zmap = np.zeros(T.n_zc, dtype=np.int64)
    for z in range(T.n_zc):
        zmap[z] = (z % (d - 1)) * d + z // (d - 1)
    for v in range(T.n_q):
        zs = sorted(int(zmap[x]) for x in T.qz[v] if x >= 0)
        xs = sorted(int(x) for x in T.qx[perm[v]] if x >= 0)
        assert zs == xs, (v, zs, xs)
    assert sorted(perm.tolist()) == list(range(T.n_q))
    if not with_xmap:
        return perm, zmap, np.array(col0, dtype=np.int64)
    xmap = np.zeros(T.n_xc, dtype=np.int64)
    for x in range(T.n_xc):
        xmap[x] = (x % d) * (d - 1) + x // d
    for v in range(T.n_q):
        xs = sorted(int(xmap[x]) for x in T.qx[v] if x >= 0)
        zs = sorted(int(z) for z in T.qz[perm[v]] if z >= 0)
        assert xs == zs, (v, xs, zs)
    return perm, zmap, xmap, np.array(col0, dtype=np.int64)


def x_part_observable(T, col0, p, seed, shot0, n):
    """Parity of the X component of the depolarizing draw over the qubits of
    data column 0 (the support of a Z logical), per shot: bit planes [W]."""
    t1 = int(oracle.threshold(np.array([p / 3.0]))[0])
    t2 = int(oracle.threshold(np.array([2.0 * p / 3.0]))[0])
    W = (n + 63) // 64
    par = np.zeros(n, dtype=np.uint8)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    sig = shot0 + np.arange(n, dtype=np.uint64)
    for v in col0:
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = v
        ctr[:, 1] = (sig & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        ctr[:, 2] = (sig >> np.uint64(32)).astype(np.uint32)
        ctr[:, 3] = DEPOL_TAG
        u = oracle.philox(ctr, np.tile(key, (n, 1)))[:, 0]
        par ^= (u < t2).astype(np.uint8)            # X or Y
    bits = np.zeros(W * 64, dtype=np.uint8)
    bits[:n] = par
    return np.packbits(bits, bitorder="little").view(np.uint64)


def run_point(d, p, n, T_iters, variant, readings, seed, threads=None):
    dem = oracle.code_capacity(d, p, unrotated=True)
    tab = oracle.tables(dem)
    tn = oracle.tanner(d, dem, unrotated=True)
    perm, zmap, col0 = transposition(d, tn)
    synx, synz, obs_z = oracle.sample_depolarizing(tn, p, seed, 0, n)
    syn_xp = np.zeros_like(synx)
    syn_xp[zmap] = synz
    obs_x = x_part_observable(tn, col0, p, seed, 0, n)
    out = {}
    for r in readings:
        kw = dict(variant=variant, threads=threads)
        iters = T_iters
        if r == "xz-lit":
            iters = (T_iters + 1) // 2
        if r == "xz-blk":
            kw["fc_rule"] = 1
        if r == "xz-xor":
            kw["weight_rule"] = 1
        rz = oracle.decode(dem, tab, synx, obs_z, n, iters, **kw)
        fz = rz.fail
        ncz = (rz.s >= 2) & ((rz.flags & oracle.F_CONVERGED_ANY) == 0)
        if r == "z":
            out[r] = (float(fz.mean()), float(ncz.mean()))
            continue
        rx = oracle.decode(dem, tab, syn_xp, obs_x, n, iters, **kw)
        ncx = (rx.s >= 2) & ((rx.flags & oracle.F_CONVERGED_ANY) == 0)
        out[r] = (float((fz | rx.fail).mean()), float((ncz | ncx).mean()))
    return out


def bbp4mf_point(d, p, n, seed, threads=None):
    """B-BP4MF (T = 25 + 25) logical error rates (z, xz) of one depolarizing
    draw: the Z part as the library decodes it, and either part failing, the
    X part decoded as the Z part of the transposed instance (the code and the
    depolarizing channel are symmetric under the transposition with X and Z
    exchanged, so the quaternary BP of the transposed instance is that of the
    original with the two Pauli components swapped)."""
    dem = oracle.code_capacity(d, p, unrotated=True)
    tn = oracle.tanner(d, dem, unrotated=True)
    perm, zmap, xmap, col0 = transposition(d, tn, with_xmap=True)
    synx, synz, obs_z = oracle.sample_depolarizing(tn, p, seed, 0, n)
    syn_xp = np.zeros_like(synx)
    syn_xp[zmap] = synz
    syn_zp = np.zeros_like(synz)
    syn_zp[xmap] = synx
    obs_x = x_part_observable(tn, col0, p, seed, 0, n)
    rz = oracle.bbp4mf_decode(dem, tn, p, synx, synz, obs_z, n, 25, threads=threads)
    rx = oracle.bbp4mf_decode(dem, tn, p, syn_xp, syn_zp, obs_x, n, 25, threads=threads)
    return float(rz.fail.mean()), float((rz.fail | rx.fail).mean())


def bbp4mf_study(n, threads):
    """B-BP4MF against the paper's printed code-capacity panel."""
    pt = {}
    for ln in open(os.path.join(ROOT, "tests", "golden", "paper_bbp4mf_code_capacity_unrotated.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        d, p, v = ln.split()
        pt[(int(d), round(float(p), 2))] = float(v)
    t0 = time.time()
    ps = (0.05, 0.08, 0.10, 0.12, 0.14, 0.16, 0.18)
    print("## B-BP4MF, unrotated code, code capacity, T = 25 + 25, %d shots per point\n" % n)
    print("| d | reading | " + " | ".join("%.2f" % p for p in ps) + " |")
    print("|---|---|" + "---|" * len(ps))
    for d in (5, 9, 13):
        rows = {"z": [], "xz": []}
        for p in ps:
            z, xz = bbp4mf_point(d, p, n, 0x2603_0538_0D00 + 100 * d + int(round(p * 100)), threads)
            rows["z"].append(z)
            rows["xz"].append(xz)
        print("| %d | paper | " % d + " | ".join("%.4f" % pt[(d, p)] for p in ps) + " |")
        for k in ("z", "xz"):
            print("| %d | %s | " % (d, k) + " | ".join("%.4f" % x for x in rows[k]) + " |", flush=True)
    print("\n(%.0f s)\n" % (time.time() - t0))


def threshold_study(n, threads):
    """Crossings of the xz logical error rate curves, BP4M and BP4MF."""
    t0 = time.time()
    for vname, variant in (("BP4M", 0), ("BP4MF", 1)):
        print("## %s, xz reading, unrotated code, code capacity, T = 25, %d shots per point\n" % (vname, n))
        ps = (0.10, 0.11, 0.12, 0.13, 0.14, 0.15)
        print("| d | " + " | ".join("%.2f" % p for p in ps) + " |")
        print("|---|" + "---|" * len(ps))
        for d in (5, 9, 13):
            row = []
            for p in ps:
                r = run_point(d, p, n, 25, variant, ("xz",), 0x2603_0538_0C00 + 100 * d + int(p * 100), threads)
                row.append(r["xz"][0])
            print("| %d | " % d + " | ".join("%.4f" % x for x in row) + " |", flush=True)
        print("\n(%.0f s)\n" % (time.time() - t0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer shots per point")
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--threshold", type=int, default=0, metavar="SHOTS",
                    help="instead: BP4M and BP4MF logical error rates under the xz reading at "
                         "d in {5, 9, 13}, p = 0.10 .. 0.15 (the threshold region), SHOTS per point")
    ap.add_argument("--bbp4mf", type=int, default=0, metavar="SHOTS",
                    help="instead: B-BP4MF logical error rates (Z part, and either part) next to the paper's "
                         "printed code-capacity panel, d in {5, 9, 13}, SHOTS per point")
    args = ap.parse_args()
    if args.bbp4mf:
        bbp4mf_study(args.bbp4mf, args.threads)
        return
    if args.threshold:
        threshold_study(args.threshold, args.threads)
        return
    scale = 0.1 if args.quick else 1.0
    pt = paper_tables()
    t0 = time.time()

    # fraction of BP4M shots never converged (the paper's "calls to MWPM")
    print("## BP4M never-converged fraction, unrotated code, code capacity, T = 25\n")
    print("| d | p | paper | z | xz | xz-lit | shots |")
    print("|---|---|---|---|---|---|---|")
    for d in (3, 5, 7, 9, 11):
        for p in (0.02, 0.06, 0.10, 0.14):
            n = int((20_000 if p < 0.05 else 6_000) * scale)
            r = run_point(d, p, n, 25, 0, ("z", "xz", "xz-lit"), 0x2603_0538_0A00 + 100 * d + int(p * 100),
                          args.threads)
            print("| %d | %.2f | %.4f | %.4f | %.4f | %.4f | %d |" % (
                d, p, pt[("rnc", d, round(p, 2))], r["z"][1], r["xz"][1], r["xz-lit"][1], n), flush=True)
    print("\n(%.0f s)\n" % (time.time() - t0))

    # logical error rates at d = 9 and 11
    for vname, variant, reads in (("BP4M", 0, ("z", "xz", "xz-lit")),
                                  ("BP4MF", 1, ("z", "xz", "xz-lit", "xz-blk", "xz-xor"))):
        print("## %s logical error rate, unrotated code, code capacity, T = 25\n" % vname)
        print("| d | p | paper | MWPM (paper) | " + " | ".join(reads) + " | shots |")
        print("|---|---|---|---|" + "---|" * len(reads) + "---|")
        for d in (9, 11):
            for p in (0.02, 0.05, 0.10, 0.15):
                n = int({0.02: 200_000, 0.05: 60_000, 0.10: 12_000, 0.15: 6_000}[p] * scale)
                r = run_point(d, p, n, 25, variant, reads, 0x2603_0538_0B00 + 100 * d + int(p * 100), args.threads)
                print("| %d | %.2f | %.3g | %.3g | " % (d, p, pt[("ler_" + vname.lower(), d, round(p, 2))],
                                                       pt[("ler_mwpm", d, round(p, 2))]) +
                      " | ".join("%.3g" % r[k][0] for k in reads) + " | %d |" % n, flush=True)
        print("\n(%.0f s)\n" % (time.time() - t0))


if __name__ == "__main__":
    main()
