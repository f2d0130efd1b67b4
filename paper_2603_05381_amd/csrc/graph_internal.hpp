// Host-side detector graphs and path tables of the bpm library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bpm.h"

namespace bpm {

// Error mechanisms in CSR form: mechanism m flips dets[off[m]..off[m+1])
// and the observable iff obs[m]; it fires with probability q[m].
struct MechanismList {
    int32_t n_det = 0;
    std::vector<int32_t> off{0};
    std::vector<int32_t> dets;
    std::vector<uint8_t> obs;
    std::vector<double> q;
    int32_t size() const { return static_cast<int32_t>(q.size()); }
};

// N x N path tables; entry [u][u] is u's path to the boundary.
struct PathTables {
    int32_t n = 0;
    std::vector<int64_t> dist;   // fixed point, 2^-32 units
    std::vector<int32_t> hops;
    std::vector<uint8_t> par;
    std::vector<int32_t> pred;   // edge id of the last edge of the path
    std::vector<double> llr;     // prior log-likelihood ratio
};

// Tanner graph of a code-capacity code with both check types (B-BP4MF):
// qc[4v..] = qubit v's X checks then Z checks (id n_xc + z), ascending, -1
// padded; cq[4c..] = check c's qubits ascending; cs[4c..] = c's slot in those
// qubits' lists; qobs[v] = a Z error on v flips the observable; qmech[v] = the
// mechanism (decoding-graph edge) that is v's Z error; noff / nedge = the
// decoding graph's edges at node u (node n_det = the boundary), ascending.
struct TannerHost {
    int32_t n_q = 0, n_xc = 0, n_zc = 0;
    std::vector<int32_t> qc, cq, cs, qmech, noff, nedge;
    std::vector<uint8_t> qobs;
};

// Returns an empty string on success, else the reason.
std::string build_code_capacity(int d, double p, MechanismList &out);
std::string build_code_capacity_unrotated(int d, double p, MechanismList &out);
std::string build_memory_z(int d, int rounds, double p, MechanismList &out);
std::string build_memory_z_unrotated(int d, int rounds, double p, MechanismList &out);
std::string build_path_tables(const MechanismList &m, PathTables &out);
std::string build_tanner_code_capacity(int d, bool unrotated, const MechanismList &m, TannerHost &t);

// Records msg as this thread's bpm_last_error() and returns st.
bpm_status set_last_error(bpm_status st, const std::string &msg);

int64_t fixed_point_weight(double q);
double prior_llr(int64_t dist_fixed);
uint32_t fire_threshold(double q);

}  // namespace bpm
