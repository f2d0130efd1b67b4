"""Pins of the readings study's own pieces (oracle/readings.py): the
transposition that decodes the X part of a depolarizing draw on the Z-error
graph, and the per-qubit redraw of the depolarizing sample that gives the X
part's observable.

 - Every qubit's Z checks, mapped by the transposition, are its image's X
   checks (checked inside readings.transposition, here for d = 2..9).
 - Redrawing the Z component over the X logical's qubits with the same
   counter layout gives the sampler's observable planes bit for bit, so the
   same redraw of the X component over the Z logical's qubits is the X
   part's observable.
 - The X part's syndrome (Z checks, from the sampler) mapped to X-check order
   equals the syndrome of the transposed X component, computed here from the
   redraw of every qubit; for B-BP4MF, which reads both syndromes, the Z
   part's syndrome (X checks) mapped to Z-check order equals that of the
   transposed Z component as well.
"""
import numpy as np
import pytest

import oracle
from oracle import readings


@pytest.mark.parametrize("d", [2, 3, 5, 9])
def test_transposition_maps_z_checks_to_x_checks(d):
    dem = oracle.code_capacity(d, 0.1, unrotated=True)
    tn = oracle.tanner(d, dem, unrotated=True)
    perm, zmap, col0 = readings.transposition(d, tn)
    assert len(col0) == d and sorted(zmap.tolist()) == list(range(tn.n_zc))
    perm2, zmap2, xmap, col02 = readings.transposition(d, tn, with_xmap=True)
    assert np.array_equal(perm, perm2) and np.array_equal(zmap, zmap2)
    assert sorted(xmap.tolist()) == list(range(tn.n_xc))
    # transposing twice is the identity on qubits and on checks
    assert np.array_equal(perm[perm], np.arange(tn.n_q))
    assert np.array_equal(xmap[zmap], np.arange(tn.n_zc)) and np.array_equal(zmap[xmap], np.arange(tn.n_xc))


def _redraw(tn, p, seed, n):
    """Pauli code per (qubit, shot): 0 I, 1 X, 2 Y, 3 Z, as the sampler draws it."""
    t1, t2, t3 = (int(oracle.threshold(np.array([k * p / 3.0]))[0]) for k in (1, 2, 3))
    E = np.zeros((tn.n_q, n), dtype=np.uint8)
    key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32), (n, 1))
    for v in range(tn.n_q):
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = v
        ctr[:, 1] = np.arange(n, dtype=np.uint32)
        ctr[:, 3] = readings.DEPOL_TAG
        u = oracle.philox(ctr, key)[:, 0].astype(np.int64)
        E[v] = np.where(u < t1, 1, np.where(u < t2, 2, np.where(u < t3, 3, 0)))
    return E


def _planes(bits):
    n = bits.shape[-1]
    W = (n + 63) // 64
    pad = np.zeros(bits.shape[:-1] + (W * 64,), dtype=np.uint8)
    pad[..., :n] = bits
    return np.packbits(pad, axis=-1, bitorder="little").view(np.uint64)


@pytest.mark.parametrize("d,p", [(3, 0.15), (5, 0.1)])
def test_redraw_reproduces_the_sampler_and_the_x_part(d, p):
    dem = oracle.code_capacity(d, p, unrotated=True)
    tn = oracle.tanner(d, dem, unrotated=True)
    perm, zmap, col0 = readings.transposition(d, tn)
    n, seed = 3000, 991
    synx, synz, obs = oracle.sample_depolarizing(tn, p, seed, 0, n)
    E = _redraw(tn, p, seed, n)
    zc = (E >= 2).astype(np.uint8)                   # Z component
    xc = ((E == 1) | (E == 2)).astype(np.uint8)      # X component
    assert np.array_equal(_planes((zc[tn.qobs == 1].sum(axis=0) & 1).astype(np.uint8)), obs)
    assert np.array_equal(readings.x_part_observable(tn, col0, p, seed, 0, n),
                          _planes((xc[col0].sum(axis=0) & 1).astype(np.uint8)))
    # syndrome of the transposed X component on the X checks
    xt = np.zeros_like(xc)
    xt[perm] = xc
    syn_t = np.zeros((tn.n_xc, n), dtype=np.uint8)
    for v in range(tn.n_q):
        for c in tn.qx[v]:
            if c >= 0:
                syn_t[c] ^= xt[v]
    mapped = np.zeros_like(synx)
    mapped[zmap] = synz
    assert np.array_equal(mapped, _planes(syn_t))
    # and its observable under the transposition is the X part's
    assert np.array_equal(_planes((xt[tn.qobs == 1].sum(axis=0) & 1).astype(np.uint8)),
                          readings.x_part_observable(tn, col0, p, seed, 0, n))
    # the transposed Z component's syndrome on the Z checks is the Z part's
    # syndrome (X checks) in Z-check order
    _, _, xmap, _ = readings.transposition(d, tn, with_xmap=True)
    zt = np.zeros_like(zc)
    zt[perm] = zc
    syn_tz = np.zeros((tn.n_zc, n), dtype=np.uint8)
    for v in range(tn.n_q):
        for c in tn.qz[v]:
            if c >= 0:
                syn_tz[c] ^= zt[v]
    mapped_z = np.zeros_like(synz)
    mapped_z[xmap] = synx
    assert np.array_equal(mapped_z, _planes(syn_tz))
