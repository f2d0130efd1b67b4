// Detector graphs of the rotated surface code and their decoding-graph path
// tables (host side of bpm_build_graph).
//
// Lattice.  Data qubit (r, c), 0 <= r, c < d, is qubit r*d + c.  The face
// (r, c), -1 <= r, c <= d-1, touches the data corners (r,c) (r,c+1) (r+1,c)
// (r+1,c+1) inside the lattice; it is an X face when r + c is even.  Interior
// faces are all stabilizers; on the top and bottom rows only X faces are, on
// the left and right columns only Z faces; corner faces never.  Stabilizers
// of a type are numbered row-major in (r, c).
//
// Code capacity (Sec. I.B, Sec. III.E): one mechanism per data qubit (Z
// error, probability 2p/3) flipping the X stabilizers that touch it; the
// observable is its overlap with the X logical on column 0.
//
// Memory-Z circuit (Sec. III.E): reset everything (flip p), then per round:
// depolarize the data, H on X ancillas (+depolarize), four CNOT layers with
// X faces visiting corners TL, TR, BL, BR and Z faces TL, BL, TR, BR (each
// followed by two-qubit depolarizing noise), H on X ancillas (+depolarize),
// flip-measure-reset-flip the ancillas; finally flip and measure the data.
// Detectors: Z stabilizers per round (vs. the previous round) and at the
// final readout; observable: Z logical on data row 0.  The unrotated code's
// memory-Z circuit is the same sequence on its own layout (see
// build_memory_z_unrotated).
//
// Fault symptoms are found by propagating every detector BACKWARD through
// the circuit as a Pauli observable (the Heisenberg picture): an error at a
// point flips exactly the detectors whose back-propagated observable it
// anticommutes with.  All detectors travel together as bit sets.
//
// Channels -> independent mechanisms: each non-identity Pauli of a k-qubit
// depolarizing channel fires independently with q, (1-2q)^(4^k/2) =
// 1 - 4^k p/(4^k - 1); an X flip fires with p.  Faults with the same
// (detectors, observable) merge as independent events: 1 - 2q = product of
// (1 - 2q_i), taken class by class (flips, 1-qubit, 2-qubit).  Mechanisms
// are ordered by (detector list, observable), lexicographically.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <queue>
#include <thread>
#include <tuple>

#include "graph_internal.hpp"

namespace bpm {
namespace {

struct Lattice {
    int d;
    std::vector<int> xid, zid;                 // (r+1)*(d+1)+(c+1) -> index or -1
    std::vector<std::pair<int, int>> xf, zf;   // faces in index order

    explicit Lattice(int d_) : d(d_), xid((d_ + 1) * (d_ + 1), -1), zid((d_ + 1) * (d_ + 1), -1) {
        for (int r = -1; r <= d - 1; ++r)
            for (int c = -1; c <= d - 1; ++c) {
                bool edge_row = (r == -1 || r == d - 1);
                bool edge_col = (c == -1 || c == d - 1);
                if (edge_row && edge_col) continue;
                bool xface = ((r + c) % 2 + 2) % 2 == 0;
                if (xface && !edge_col) { xid[slot(r, c)] = (int)xf.size(); xf.push_back({r, c}); }
                if (!xface && !edge_row) { zid[slot(r, c)] = (int)zf.size(); zf.push_back({r, c}); }
            }
    }
    int slot(int r, int c) const { return (r + 1) * (d + 1) + (c + 1); }
    bool inside(int r, int c) const { return r >= 0 && r < d && c >= 0 && c < d; }
    int xface(int r, int c) const {
        if (r < -1 || r > d - 1 || c < -1 || c > d - 1) return -1;
        return xid[slot(r, c)];
    }
};

enum OpKind : uint8_t { kReset, kHad, kCnot, kMeasure, kDep1, kDep2, kFlip };
struct Op { OpKind kind; int a, b; };

// Bit set over the detectors plus one trailing bit for the observable.
using Bits = std::vector<uint64_t>;

inline void bxor(Bits &a, const Bits &b) { for (size_t i = 0; i < a.size(); ++i) a[i] ^= b[i]; }

using Key = std::pair<std::vector<int32_t>, int>;

}  // namespace

int64_t fixed_point_weight(double q) {
    double w = std::log((1.0 - q) / q);
    long long f = std::llround(w * 4294967296.0);
    return f < 1 ? 1 : (int64_t)f;
}

double prior_llr(int64_t dist_fixed) {
    double D = std::ldexp((double)dist_fixed, -32);
    double e = std::exp(-D);
    double t = std::log1p(-e);
    return (-D) - t;
}

uint32_t fire_threshold(double q) {
    double t = std::floor(q * 4294967296.0 + 0.5);
    if (t < 0.0) t = 0.0;
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

std::string build_code_capacity(int d, double p, MechanismList &out) {
    if (d < 3 || d % 2 == 0) return "code distance must be odd and >= 3";
    if (!(p > 0.0 && p < 0.75)) return "code-capacity p must lie in (0, 0.75)";
    Lattice L(d);
    out = MechanismList();
    out.n_det = (int32_t)L.xf.size();
    const double q = (2.0 * p) / 3.0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            std::vector<int32_t> ds;
            for (int dr = -1; dr <= 0; ++dr)
                for (int dc = -1; dc <= 0; ++dc) {
                    int id = L.xface(r + dr, c + dc);
                    if (id >= 0) ds.push_back(id);
                }
            std::sort(ds.begin(), ds.end());
            out.dets.insert(out.dets.end(), ds.begin(), ds.end());
            out.off.push_back((int32_t)out.dets.size());
            out.obs.push_back(c == 0 ? 1 : 0);
            out.q.push_back(q);
        }
    return "";
}

// Unrotated (planar) surface code, code capacity.  On the (2d-1) x (2d-1)
// grid, data qubits sit at (r, c) with r + c even, X stabilizers at (r odd,
// c even) (numbered ((r-1)/2)*d + c/2) and Z stabilizers at (r even, c odd).
// A Z error on a data qubit flips the X stabilizers above/below it (c even)
// or left/right of it (c odd); qubits of rows 0 and 2d-2 touch one X
// stabilizer and connect to the boundary.  The X logical runs along data
// row 0, so a Z error there flips the observable.  Mechanisms are listed in
// the canonical order (detector tuple, then observable).
std::string build_code_capacity_unrotated(int d, double p, MechanismList &out) {
    if (d < 2) return "code distance must be >= 2";
    if (!(p > 0.0 && p < 0.75)) return "code-capacity p must lie in (0, 0.75)";
    const int n = 2 * d - 1;
    auto xcheck = [&](int r, int c) -> int {
        if (r < 0 || r >= n || c < 0 || c >= n || (r & 1) == 0 || (c & 1) != 0) return -1;
        return ((r - 1) / 2) * d + c / 2;
    };
    struct M { std::vector<int32_t> dets; uint8_t obs; };
    std::vector<M> ms;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            if ((r + c) & 1) continue;
            M m;
            const int nb[4][2] = {{r - 1, c}, {r + 1, c}, {r, c - 1}, {r, c + 1}};
            for (auto &x : nb) {
                const int id = xcheck(x[0], x[1]);
                if (id >= 0) m.dets.push_back(id);
            }
            std::sort(m.dets.begin(), m.dets.end());
            m.obs = r == 0 ? 1 : 0;
            ms.push_back(std::move(m));
        }
    std::sort(ms.begin(), ms.end(), [](const M &a, const M &b) {
        if (a.dets != b.dets) return std::lexicographical_compare(a.dets.begin(), a.dets.end(), b.dets.begin(), b.dets.end());
        return a.obs < b.obs;
    });
    out = MechanismList();
    out.n_det = d * (d - 1);
    const double q = (2.0 * p) / 3.0;
    for (const M &m : ms) {
        out.dets.insert(out.dets.end(), m.dets.begin(), m.dets.end());
        out.off.push_back((int32_t)out.dets.size());
        out.obs.push_back(m.obs);
        out.q.push_back(q);
    }
    return "";
}

namespace {

// Qubits and CNOT schedule of one memory-Z round: data qubits 0..nd-1, then
// the X ancillas, then the Z ancillas.  In CNOT layer k, X stabilizer i acts
// on data xcnot[i][k] (ancilla as control) and Z stabilizer i on zcnot[i][k]
// (ancilla as target); -1 = no qubit there.  zsupp lists each Z
// stabilizer's data qubits (for the final detectors), obs_data the data
// qubits whose Z readouts form the logical observable.
struct MemoryLayout {
    int nd = 0, nx = 0, nz = 0;
    std::vector<std::array<int, 4>> xcnot, zcnot;
    std::vector<std::vector<int>> zsupp;
    std::vector<int> obs_data;
};

std::string build_memory_circuit(const MemoryLayout &Y, int rounds, double p, MechanismList &out);

}  // namespace

std::string build_memory_z(int d, int rounds, double p, MechanismList &out) {
    if (d < 3 || d % 2 == 0) return "code distance must be odd and >= 3";
    if (rounds < 1) return "rounds must be >= 1";
    if (!(p > 0.0 && p < 0.5)) return "circuit-level p must lie in (0, 0.5)";
    Lattice L(d);
    MemoryLayout Y;
    Y.nd = d * d;
    Y.nx = (int)L.xf.size();
    Y.nz = (int)L.zf.size();
    static const int xorder[4][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
    static const int zorder[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (int i = 0; i < Y.nx; ++i) {
        std::array<int, 4> a;
        for (int k = 0; k < 4; ++k) {
            const int r = L.xf[i].first + xorder[k][0], c = L.xf[i].second + xorder[k][1];
            a[k] = L.inside(r, c) ? r * d + c : -1;
        }
        Y.xcnot.push_back(a);
    }
    for (int i = 0; i < Y.nz; ++i) {
        std::array<int, 4> a;
        std::vector<int> sup;
        for (int k = 0; k < 4; ++k) {
            const int r = L.zf[i].first + zorder[k][0], c = L.zf[i].second + zorder[k][1];
            a[k] = L.inside(r, c) ? r * d + c : -1;
            if (a[k] >= 0) sup.push_back(a[k]);
        }
        Y.zcnot.push_back(a);
        Y.zsupp.push_back(sup);
    }
    for (int c = 0; c < d; ++c) Y.obs_data.push_back(c);
    return build_memory_circuit(Y, rounds, p, out);
}

// Unrotated (planar) code, memory-Z.  Grid of the code-capacity builder:
// data at (r, c), r + c even, numbered row-major; X stabilizers at (r odd,
// c even), Z stabilizers at (r even, c odd), each numbered row-major.  CNOT
// layers visit the neighbours N, W, E, S (X stabilizers) and N, E, W, S (Z
// stabilizers): in every layer both types move along the same axis, so no
// data qubit is used twice, and each X / Z pair sharing two data qubits
// visits both in the same relative order, so every detector is
// deterministic.  An ancilla X error before the last two CNOTs of an X
// stabilizer leaves X on its E and S neighbours, one vertical and one
// horizontal edge of the Z-detector graph meeting at a node, which advances
// a left-right chain by one column like a single edge, so the circuit keeps
// distance d.  The Z-detector graph's boundaries are the left and right data
// columns; the observable is the Z readout of data column 0.
std::string build_memory_z_unrotated(int d, int rounds, double p, MechanismList &out) {
    if (d < 2) return "code distance must be >= 2";
    if (rounds < 1) return "rounds must be >= 1";
    if (!(p > 0.0 && p < 0.5)) return "circuit-level p must lie in (0, 0.5)";
    const int n = 2 * d - 1;
    auto data = [&](int r, int c) -> int {
        if (r < 0 || r >= n || c < 0 || c >= n || ((r + c) & 1)) return -1;
        return (r / 2) * (2 * d - 1) + ((r & 1) ? d + (c - 1) / 2 : c / 2);
    };
    static const int xdir[4][2] = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};   // N W E S
    static const int zdir[4][2] = {{-1, 0}, {0, 1}, {0, -1}, {1, 0}};   // N E W S
    MemoryLayout Y;
    Y.nd = d * d + (d - 1) * (d - 1);
    for (int r = 1; r < n; r += 2)
        for (int c = 0; c < n; c += 2) {
            std::array<int, 4> a;
            for (int k = 0; k < 4; ++k) a[k] = data(r + xdir[k][0], c + xdir[k][1]);
            Y.xcnot.push_back(a);
        }
    for (int r = 0; r < n; r += 2)
        for (int c = 1; c < n; c += 2) {
            std::array<int, 4> a;
            std::vector<int> sup;
            for (int k = 0; k < 4; ++k) {
                a[k] = data(r + zdir[k][0], c + zdir[k][1]);
                if (a[k] >= 0) sup.push_back(a[k]);
            }
            Y.zcnot.push_back(a);
            Y.zsupp.push_back(sup);
        }
    Y.nx = (int)Y.xcnot.size();
    Y.nz = (int)Y.zcnot.size();
    for (int r = 0; r < n; r += 2) Y.obs_data.push_back(data(r, 0));
    return build_memory_circuit(Y, rounds, p, out);
}

namespace {

// Reset everything (flip p), then per round: depolarize the data, H on the
// X ancillas (+depolarize), the four CNOT layers (each followed by two-qubit
// depolarizing noise), H on the X ancillas (+depolarize), flip-measure-
// reset-flip the ancillas; finally flip and measure the data.  Detectors: Z
// stabilizers per round (vs. the previous round) and at the final readout.
std::string build_memory_circuit(const MemoryLayout &Y, int rounds, double p, MechanismList &out) {
    const int nd = Y.nd, nx = Y.nx, nz = Y.nz;
    const int nq = nd + nx + nz;
    auto xanc = [&](int i) { return nd + i; };
    auto zanc = [&](int i) { return nd + nx + i; };

    // ---- circuit ----
    std::vector<Op> ops;
    int n_rec = 0;
    std::vector<int> zrec((size_t)rounds * nz), drec(nd);
    for (int q = 0; q < nq; ++q) { ops.push_back({kReset, q, 0}); ops.push_back({kFlip, q, 0}); }
    for (int t = 0; t < rounds; ++t) {
        for (int q = 0; q < nd; ++q) ops.push_back({kDep1, q, 0});
        for (int i = 0; i < nx; ++i) { ops.push_back({kHad, xanc(i), 0}); ops.push_back({kDep1, xanc(i), 0}); }
        for (int k = 0; k < 4; ++k) {
            std::vector<std::pair<int, int>> layer;
            for (int i = 0; i < nx; ++i)
                if (Y.xcnot[i][k] >= 0) layer.push_back({xanc(i), Y.xcnot[i][k]});
            for (int i = 0; i < nz; ++i)
                if (Y.zcnot[i][k] >= 0) layer.push_back({Y.zcnot[i][k], zanc(i)});
            for (auto &g : layer) ops.push_back({kCnot, g.first, g.second});
            for (auto &g : layer) ops.push_back({kDep2, g.first, g.second});
        }
        for (int i = 0; i < nx; ++i) { ops.push_back({kHad, xanc(i), 0}); ops.push_back({kDep1, xanc(i), 0}); }
        for (int q = nd; q < nq; ++q) ops.push_back({kFlip, q, 0});
        for (int q = nd; q < nq; ++q) {
            if (q >= nd + nx) zrec[(size_t)t * nz + (q - nd - nx)] = n_rec;
            ops.push_back({kMeasure, q, n_rec++});
        }
        for (int q = nd; q < nq; ++q) { ops.push_back({kReset, q, 0}); ops.push_back({kFlip, q, 0}); }
    }
    for (int q = 0; q < nd; ++q) ops.push_back({kFlip, q, 0});
    for (int q = 0; q < nd; ++q) { drec[q] = n_rec; ops.push_back({kMeasure, q, n_rec++}); }

    // ---- detectors as sets of measurement records ----
    const int n_det = (rounds + 1) * nz;
    const int nbits = n_det + 1, nw = (nbits + 63) / 64;
    std::vector<Bits> rec_dets(n_rec, Bits(nw, 0));
    auto add = [&](int rec, int bit) { rec_dets[rec][bit >> 6] ^= 1ull << (bit & 63); };
    for (int t = 0; t < rounds; ++t)
        for (int i = 0; i < nz; ++i) {
            add(zrec[(size_t)t * nz + i], t * nz + i);
            if (t > 0) add(zrec[(size_t)(t - 1) * nz + i], t * nz + i);
        }
    for (int i = 0; i < nz; ++i) {
        int det = rounds * nz + i;
        add(zrec[(size_t)(rounds - 1) * nz + i], det);
        for (int q : Y.zsupp[i]) add(drec[q], det);
    }
    for (int q : Y.obs_data) add(drec[q], n_det);

    // ---- backward sweep ----
    std::vector<Bits> ox(nq, Bits(nw, 0)), oz(nq, Bits(nw, 0));
    const double fflip = 1.0 - 2.0 * p;
    const double f1 = std::sqrt(1.0 - (4.0 * p) / 3.0);
    const double f2 = std::sqrt(std::sqrt(std::sqrt(1.0 - (16.0 * p) / 15.0)));
    std::map<Key, std::array<int, 3>> merged;
    int gauge_bad = 0;
    auto is_zero = [](const Bits &b) { for (uint64_t w : b) if (w) return false; return true; };
    auto record = [&](const Bits &sym, int cls) {
        std::vector<int32_t> ds;
        for (int w = 0; w < nw; ++w) {
            uint64_t v = sym[w];
            while (v) {
                int b = __builtin_ctzll(v);
                v &= v - 1;
                int bit = w * 64 + b;
                if (bit < n_det) ds.push_back(bit);
            }
        }
        int ob = (int)((sym[n_det >> 6] >> (n_det & 63)) & 1);
        if (ds.empty() && !ob) return;
        merged[Key(std::move(ds), ob)][cls]++;
    };
    Bits tmp(nw);
    for (size_t i = ops.size(); i-- > 0;) {
        const Op &o = ops[i];
        switch (o.kind) {
        case kReset:
            if (!is_zero(ox[o.a])) ++gauge_bad;   // Z right after a reset must be harmless
            std::fill(ox[o.a].begin(), ox[o.a].end(), 0);
            std::fill(oz[o.a].begin(), oz[o.a].end(), 0);
            break;
        case kMeasure:
            if (!is_zero(ox[o.a])) ++gauge_bad;   // Z right after a readout must be harmless
            bxor(oz[o.a], rec_dets[o.b]);
            break;
        case kHad:
            std::swap(ox[o.a], oz[o.a]);
            break;
        case kCnot:
            bxor(oz[o.a], oz[o.b]);
            bxor(ox[o.b], ox[o.a]);
            break;
        case kFlip:
            record(oz[o.a], 0);
            break;
        case kDep1:
            record(oz[o.a], 1);                        // X
            record(ox[o.a], 1);                        // Z
            tmp = oz[o.a]; bxor(tmp, ox[o.a]);
            record(tmp, 1);                            // Y
            break;
        case kDep2: {
            const Bits *g[4] = {&oz[o.a], &ox[o.a], &oz[o.b], &ox[o.b]};  // X_a Z_a X_b Z_b
            for (int mask = 1; mask < 16; ++mask) {
                std::fill(tmp.begin(), tmp.end(), 0);
                for (int k = 0; k < 4; ++k) if (mask >> k & 1) bxor(tmp, *g[k]);
                record(tmp, 2);
            }
            break;
        }
        }
    }
    if (gauge_bad) return "internal error: non-deterministic detector in the memory-Z circuit";

    out = MechanismList();
    out.n_det = n_det;
    for (auto &kv : merged) {
        const auto &ds = kv.first.first;
        if (ds.empty()) return "internal error: undetectable logical error mechanism";
        if (ds.size() > 2) return "memory-Z circuit produced a non-graphlike mechanism";
        double y = 1.0;
        for (int k = 0; k < kv.second[0]; ++k) y *= fflip;
        for (int k = 0; k < kv.second[1]; ++k) y *= f1;
        for (int k = 0; k < kv.second[2]; ++k) y *= f2;
        out.dets.insert(out.dets.end(), ds.begin(), ds.end());
        out.off.push_back((int32_t)out.dets.size());
        out.obs.push_back((uint8_t)kv.first.second);
        out.q.push_back(0.5 * (1.0 - y));
    }
    return "";
}

}  // namespace

// Both check types of the code-capacity codes.  Rotated: data (r, c), faces
// as in Lattice; a Z error on column-0 data flips the observable, and the
// mechanisms are listed in qubit order.  Unrotated: the grid of
// build_code_capacity_unrotated (data at r + c even, numbered row-major; X
// checks at (odd, even), Z checks at (even, odd)); a Z error on data row 0
// flips the observable; each qubit's mechanism is the one with its X checks
// and observable bit (all distinct in this layout).
std::string build_tanner_code_capacity(int d, bool unrotated, const MechanismList &m, TannerHost &t) {
    t = TannerHost();
    std::vector<std::vector<int>> xs, zs;        // per qubit
    std::vector<uint8_t> ob;
    if (unrotated) {
        const int n = 2 * d - 1;
        t.n_xc = d * (d - 1);
        t.n_zc = d * (d - 1);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                if ((r + c) & 1) continue;
                std::vector<int> x, z;
                const int nb[4][2] = {{r - 1, c}, {r + 1, c}, {r, c - 1}, {r, c + 1}};
                for (auto &q : nb) {
                    const int a = q[0], bb = q[1];
                    if (a < 0 || a >= n || bb < 0 || bb >= n) continue;
                    if ((a & 1) && !(bb & 1)) x.push_back(((a - 1) / 2) * d + bb / 2);
                    if (!(a & 1) && (bb & 1)) z.push_back((a / 2) * (d - 1) + (bb - 1) / 2);
                }
                xs.push_back(x);
                zs.push_back(z);
                ob.push_back(r == 0);
            }
    } else {
        Lattice L(d);
        t.n_xc = (int)L.xf.size();
        t.n_zc = (int)L.zf.size();
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                std::vector<int> x, z;
                for (int a = r - 1; a <= r; ++a)
                    for (int bb = c - 1; bb <= c; ++bb) {
                        if (a < -1 || a > d - 1 || bb < -1 || bb > d - 1) continue;
                        if (L.xid[L.slot(a, bb)] >= 0) x.push_back(L.xid[L.slot(a, bb)]);
                        if (L.zid[L.slot(a, bb)] >= 0) z.push_back(L.zid[L.slot(a, bb)]);
                    }
                xs.push_back(x);
                zs.push_back(z);
                ob.push_back(c == 0);
            }
    }
    const int nq = (int)xs.size(), nc = t.n_xc + t.n_zc;
    if (m.n_det != t.n_xc || m.size() != nq) return "internal error: Tanner graph does not match the detector graph";
    t.n_q = nq;
    t.qc.assign(4 * (size_t)nq, -1);
    t.cq.assign(4 * (size_t)nc, -1);
    t.cs.assign(4 * (size_t)nc, -1);
    t.qobs = ob;
    t.qmech.assign(nq, -1);
    std::map<std::pair<std::vector<int32_t>, int>, int> by_key;
    for (int e = 0; e < m.size(); ++e)
        by_key[{std::vector<int32_t>(m.dets.begin() + m.off[e], m.dets.begin() + m.off[e + 1]), m.obs[e]}] = e;
    for (int v = 0; v < nq; ++v) {
        std::sort(xs[v].begin(), xs[v].end());
        std::sort(zs[v].begin(), zs[v].end());
        if (xs[v].size() > 2 || zs[v].size() > 2) return "internal error: qubit in more than two checks of a type";
        int k = 0;
        for (int x : xs[v]) t.qc[4 * v + k++] = x;
        for (int z : zs[v]) t.qc[4 * v + k++] = t.n_xc + z;
        const std::vector<int32_t> key(xs[v].begin(), xs[v].end());
        int e = -1;
        if (unrotated) {
            auto it = by_key.find({key, ob[v]});
            if (it != by_key.end()) e = it->second;
        } else if (std::vector<int32_t>(m.dets.begin() + m.off[v], m.dets.begin() + m.off[v + 1]) == key &&
                   m.obs[v] == ob[v]) {
            e = v;
        }
        if (e < 0) return "internal error: no mechanism for a qubit's Z error";
        t.qmech[v] = e;
    }
    // every qubit has a decoding-graph edge of its own (its re-weighted
    // prior is that edge's weight)
    std::vector<char> seen(nq, 0);
    for (int v = 0; v < nq; ++v) {
        if (seen[t.qmech[v]]) return "internal error: two qubits share a decoding-graph edge";
        seen[t.qmech[v]] = 1;
    }
    std::vector<int> fill(nc, 0);
    for (int v = 0; v < nq; ++v)
        for (int k = 0; k < 4; ++k) {
            const int c = t.qc[4 * v + k];
            if (c < 0) continue;
            if (fill[c] >= 4) return "internal error: check of weight above 4";
            t.cq[4 * c + fill[c]] = v;
            t.cs[4 * c + fill[c]] = k;
            ++fill[c];
        }
    // incident edges of every decoding-graph node (boundary = node N)
    const int N = m.n_det, E = m.size();
    std::vector<std::vector<int>> inc(N + 1);
    for (int e = 0; e < E; ++e) {
        const int k = m.off[e + 1] - m.off[e];
        inc[m.dets[m.off[e]]].push_back(e);
        inc[k == 2 ? m.dets[m.off[e] + 1] : N].push_back(e);
    }
    t.noff.assign(N + 2, 0);
    for (int u = 0; u <= N; ++u) {
        t.noff[u + 1] = t.noff[u] + (int)inc[u].size();
        t.nedge.insert(t.nedge.end(), inc[u].begin(), inc[u].end());
    }
    return "";
}

// Dijkstra from every detector on (weight, hops); the boundary B = N is a
// sink.  Ties between optimal predecessors go to the smallest (node, edge),
// kept up to date during relaxation: every optimal predecessor of y is
// settled, and relaxes y, before y itself is settled.
std::string build_path_tables(const MechanismList &m, PathTables &out) {
    const int N = m.n_det, B = N, E = m.size();
    std::vector<int> eu(E), ev(E);
    std::vector<int64_t> ew(E);
    for (int e = 0; e < E; ++e) {
        int k = m.off[e + 1] - m.off[e];
        if (k < 1 || k > 2) return "decoding graph needs graphlike mechanisms";
        eu[e] = m.dets[m.off[e]];
        ev[e] = k == 2 ? m.dets[m.off[e] + 1] : B;
        ew[e] = fixed_point_weight(m.q[e]);
    }
    std::vector<std::vector<std::pair<int, int>>> adj(N + 1);   // (neighbour, edge)
    for (int e = 0; e < E; ++e) {
        adj[eu[e]].push_back({ev[e], e});
        adj[ev[e]].push_back({eu[e], e});
    }
    out = PathTables();
    out.n = N;
    const size_t NN = (size_t)N * N;
    out.dist.assign(NN, 0); out.hops.assign(NN, 0); out.par.assign(NN, 0);
    out.pred.assign(NN, -1); out.llr.assign(NN, 0.0);
    std::vector<int> failed;

    auto run = [&](int u0, int u1, int *bad) {
        std::vector<int64_t> dist(N + 1);
        std::vector<int32_t> hops(N + 1), pnode(N + 1), pedge(N + 1);
        std::vector<uint8_t> par(N + 1), settled(N + 1);
        using Item = std::tuple<int64_t, int32_t, int32_t>;
        for (int u = u0; u < u1; ++u) {
            std::fill(dist.begin(), dist.end(), INT64_MAX);
            std::fill(hops.begin(), hops.end(), INT32_MAX);
            std::fill(settled.begin(), settled.end(), 0);
            std::fill(pnode.begin(), pnode.end(), INT32_MAX);
            std::fill(pedge.begin(), pedge.end(), INT32_MAX);
            std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
            dist[u] = 0; hops[u] = 0; par[u] = 0;
            pq.push({0, 0, u});
            int n_settled = 0;
            while (!pq.empty()) {
                auto [w, h, x] = pq.top();
                pq.pop();
                if (settled[x] || w != dist[x] || h != hops[x]) continue;
                settled[x] = 1;
                ++n_settled;
                if (x != u) {
                    int e = pedge[x];
                    par[x] = par[pnode[x]] ^ m.obs[e];
                }
                if (x == B) continue;
                for (auto [y, e] : adj[x]) {
                    if (settled[y]) continue;
                    int64_t nw = w + ew[e];
                    int32_t nh = h + 1;
                    if (nw < dist[y] || (nw == dist[y] && nh < hops[y])) {
                        dist[y] = nw; hops[y] = nh; pnode[y] = x; pedge[y] = e;
                        pq.push({nw, nh, y});
                    } else if (nw == dist[y] && nh == hops[y] &&
                               (x < pnode[y] || (x == pnode[y] && e < pedge[y]))) {
                        pnode[y] = x; pedge[y] = e;
                    }
                }
            }
            if (n_settled != N + 1) { *bad = 1; return; }
            for (int v = 0; v < N; ++v) {
                int t = (v == u) ? B : v;
                size_t k = (size_t)u * N + v;
                out.dist[k] = dist[t]; out.hops[k] = hops[t]; out.par[k] = par[t];
                out.pred[k] = pedge[t]; out.llr[k] = prior_llr(dist[t]);
            }
        }
    };
    int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 32u);
    nt = std::max(1, std::min(nt, N / 16 + 1));
    std::vector<std::thread> th;
    std::vector<int> bad(nt, 0);
    for (int i = 0; i < nt; ++i)
        th.emplace_back(run, (int)((int64_t)N * i / nt), (int)((int64_t)N * (i + 1) / nt), &bad[i]);
    for (auto &t : th) t.join();
    for (int b : bad) if (b) return "detector graph is not connected to every detector";
    return "";
}

}  // namespace bpm
