// Sampling, defect extraction and result packing kernels of bpm.
//
// Sampler (detector error model of Sec. III.E): one thread per shot; every
// mechanism m fires independently iff word (m mod 4) of
// Philox4x32-10(counter = (m div 4, shot lo, shot hi, 0), key = seed) is
// below round(q_m 2^32).  Philox4x32-10 is written from its published
// definition (Salmon et al., SC'11).  A thread XORs the detectors of the
// mechanisms that fire into its own bit row in LDS (rows interleaved so that
// a wave's 64 rows sit in distinct banks); a wave then turns the 64 rows
// into detector words with one ballot per detector.  When the error planes
// are wanted, the wave also ballots every mechanism's decision and writes
// it as that mechanism's word of the 64 shots.
//
// Extraction: one thread per shot reads, detector by detector, the wave's
// 64-shot word (the same address for the whole wave) and appends the
// detectors whose bit is set, so the defect list comes out sorted.  Shots
// are binned by defect count with one atomic per wave and bin.

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_common.hpp"

namespace bpm {

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // (each 32 x 32 -> 64-bit product as one multiply-add instruction
        // rather than separate low and high multiplies)
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__global__ void k_sample(DevGraph g, uint64_t seed, uint64_t shot0, uint64_t n, uint64_t W, int nwords,
                         uint64_t *syn, uint64_t *obs, uint64_t *err) {
    extern __shared__ uint32_t rows[];          // [nwords][blockDim.x]
    const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63;
    const uint64_t b = (uint64_t)blockIdx.x * bd + tid;
    const uint64_t word = b >> 6;
    const bool active = b < n;
    for (int k = 0; k < nwords; ++k) rows[k * bd + tid] = 0u;
    const uint64_t sigma = shot0 + b;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t ob = 0;
    const int nm = g.n_mech;
    for (int m0 = 0; m0 < nm; m0 += 4) {
        uint32_t r[4];
        philox4x32_10((uint32_t)(m0 >> 2), (uint32_t)sigma, (uint32_t)(sigma >> 32), 0u, k0, k1, r);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int m = m0 + w;
            if (m >= nm) break;
            const bool fire = active && r[w] < g.thr[m];
            if (err) {                              // uniform: every lane ballots
                const uint64_t fw = __ballot(fire);
                if (lane == 0 && word < W) err[(uint64_t)m * W + word] = fw;
            }
            if (fire) {
                for (int e = g.mech_off[m]; e < g.mech_off[m + 1]; ++e) {
                    const int k = g.mech_det[e];
                    rows[(k >> 5) * bd + tid] ^= 1u << (k & 31);
                }
                ob ^= g.mech_obs[m];
            }
        }
    }
    if (word >= W) return;                      // uniform per wave
    const int N = g.n_det;
    for (int k0d = 0; k0d < N; k0d += 64) {
        uint64_t mine = 0;
        for (int j = 0; j < 64; ++j) {
            const int k = k0d + j;
            if (k >= N) break;
            const int bit = (rows[(k >> 5) * bd + tid] >> (k & 31)) & 1;
            const uint64_t bal = __ballot(bit);
            if (lane == j) mine = bal;
        }
        const int k = k0d + lane;
        if (k < N) syn[(uint64_t)k * W + word] = mine;
    }
    const uint64_t ob_word = __ballot(ob & 1u);
    if (lane == 0) obs[word] = ob_word;
}

// Depolarizing noise on every qubit of a code-capacity code with both
// syndromes (B-BP4MF input): per qubit v and shot, u = word 0 of
// Philox4x32-10(counter = (v, shot lo, shot hi, 0x44455031), key = seed)
// gives X if u < t1, Y if u < t2, Z if u < t3, else I.  The X component
// flips v's Z checks, the Z component its X checks and, on the observable's
// qubits, the observable.  Rows and ballots as in k_sample (X checks, then
// Z checks, one bit row per thread).
__global__ void k_sample_depol(TannerDev tn, uint64_t seed, uint64_t shot0, uint64_t n, uint64_t W, int nwords,
                               uint32_t t1, uint32_t t2, uint32_t t3, uint64_t *synx, uint64_t *synz,
                               uint64_t *obs) {
    extern __shared__ uint32_t rows[];          // [nwords][blockDim.x], checks 0..n_xc+n_zc-1
    const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63;
    const uint64_t b = (uint64_t)blockIdx.x * bd + tid;
    const uint64_t word = b >> 6;
    const bool active = b < n;
    for (int k = 0; k < nwords; ++k) rows[k * bd + tid] = 0u;
    const uint64_t sigma = shot0 + b;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t ob = 0;
    for (int v = 0; v < tn.n_q; ++v) {
        uint32_t r[4];
        philox4x32_10((uint32_t)v, (uint32_t)sigma, (uint32_t)(sigma >> 32), 0x44455031u, k0, k1, r);
        const uint32_t u = r[0];
        const int E = u < t1 ? 1 : u < t2 ? 2 : u < t3 ? 3 : 0;    // X, Y, Z, I
        if (!active || E == 0) continue;
        for (int k = 0; k < 4; ++k) {
            const int c = tn.qc[4 * v + k];
            if (c < 0) continue;
            const bool xcheck = c < tn.n_xc;
            // X checks see the Z component (Y, Z); Z checks the X component (X, Y)
            if (xcheck ? E >= 2 : E <= 2) rows[(c >> 5) * bd + tid] ^= 1u << (c & 31);
        }
        if (E >= 2) ob ^= tn.qobs[v];
    }
    if (word >= W) return;                      // uniform per wave
    const int nc = tn.n_xc + tn.n_zc;
    for (int c0 = 0; c0 < nc; c0 += 64) {
        uint64_t mine = 0;
        for (int j = 0; j < 64; ++j) {
            const int c = c0 + j;
            if (c >= nc) break;
            const int bit = (rows[(c >> 5) * bd + tid] >> (c & 31)) & 1;
            const uint64_t bal = __ballot(bit);
            if (lane == j) mine = bal;
        }
        const int c = c0 + lane;
        if (c < tn.n_xc) synx[(uint64_t)c * W + word] = mine;
        else if (c < nc) synz[(uint64_t)(c - tn.n_xc) * W + word] = mine;
    }
    const uint64_t ob_word = __ballot(ob & 1u);
    if (lane == 0) obs[word] = ob_word;
}

// Defect extraction for every instance of a call: one thread per shot.
// Blocks [block0, next block0) of the grid belong to one instance.
__global__ void k_extract(DecodeShared c) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int ii = block_instance(c, blockIdx.x);
    DevGraph g;
    InstState st;
    uint64_t ibase, iblock0;
    load_instance(c, ii, g, st, ibase, iblock0);
    const uint64_t b = (blockIdx.x - iblock0) * (uint64_t)blockDim.x + tid;
    const uint64_t word = b >> 6;
    if (word >= st.W) return;                   // uniform per wave
    const bool active = b < st.n_shots;
    const int N = g.n_det;
    const int cap = c.s_cap;
    uint16_t *out = st.defects + (active ? b : 0) * (uint64_t)cap;
    int s = 0;
    if (st.rows_words > 0) {
        // shot-major rows: this shot's own words, lowest detector first
        const uint64_t *row = st.syn + (active ? b : 0) * (uint64_t)st.rows_words;
        for (int w = 0; active && w < st.rows_words; ++w) {
            uint64_t x = row[w];
            while (x) {
                const int k = w * 64 + __ffsll((unsigned long long)x) - 1;
                x &= x - 1;
                if (k >= N) break;
                if (s < cap) out[s] = (uint16_t)k;
                ++s;
            }
        }
    } else {
        // bit planes: the wave's words of eight detectors are loaded
        // together (one load's latency per eight detectors instead of per
        // detector); with a row length that is a multiple of four, four
        // defects go out as one 8-byte store
        const bool pack = (cap & 3) == 0;
        uint64_t acc = 0;
        for (int k0 = 0; k0 < N; k0 += 8) {
            uint64_t w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) w[i] = k0 + i < N ? st.syn[(uint64_t)(k0 + i) * st.W + word] : 0ull;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (active && ((w[i] >> lane) & 1ull)) {
                    if (s < cap) {
                        if (pack) {
                            acc |= (uint64_t)(k0 + i) << (16 * (s & 3));
                            if ((s & 3) == 3) { *reinterpret_cast<uint64_t *>(out + (s - 3)) = acc; acc = 0; }
                        } else {
                            out[s] = (uint16_t)(k0 + i);
                        }
                    }
                    ++s;
                }
            }
        }
        if (pack) {
            const int done = s < cap ? s : cap;
            for (int r = done & ~3; r < done; ++r) out[r] = (uint16_t)(acc >> (16 * (r & 3)));
        }
    }
    int cls = -1;
    if (active) {
        st.s[b] = s;
        uint8_t fl = 0;
        if (s > cap) {
            // not decoded: counted as a logical failure, so that a logical
            // error rate over a batch with overflow is an upper bound
            fl = kOverflow | kFail;
        } else if (s <= 1) {
            fl = kConvergedAny;
            int pred = 0;
            if (s == 1) {
                const int u = out[0];
                pred = g.par[(size_t)u * N + u];
                if (st.match) st.match[b * (uint64_t)st.match_stride] = 0;
                if (st.corr) emit_path(g, u, u, st.corr, st.W, b);
            }
            const int ob = st.obs ? (int)((st.obs[word] >> lane) & 1ull) : 0;
            if (pred) fl |= kPred;
            if (pred != ob) fl |= kFail;
        } else {
            cls = class_of(s);
        }
        st.flags[b] = fl;
    }
    // wave-aggregated append to the class lists
    for (int cl = 0; cl < kClasses; ++cl) {
        const uint64_t m = __ballot(cls == cl);
        if (!m) continue;
        uint32_t base = 0;
        const int leader = __ffsll((unsigned long long)m) - 1;
        if (lane == leader) base = atomicAdd(&c.class_count[cl], (uint32_t)__popcll(m));
        base = __shfl(base, leader);
        if (cls == cl) {
            const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            c.class_list[(uint64_t)cl * c.total + base + rank] = (uint32_t)(ibase + b);
        }
    }
}

// Result packing for every instance: bit planes, per-shot copies, counters.
__global__ void k_finalize(DecodeShared c) {
    __shared__ unsigned long long acc[6];
    const int tid = threadIdx.x, lane = tid & 63;
    const int ii = block_instance(c, blockIdx.x);
    DevGraph g;
    InstState st;
    uint64_t ibase, iblock0;
    load_instance(c, ii, g, st, ibase, iblock0);
    if (tid < 6) acc[tid] = 0ull;
    __syncthreads();
    const uint64_t b = (blockIdx.x - iblock0) * (uint64_t)blockDim.x + tid;
    const uint64_t word = b >> 6;
    const bool active = b < st.n_shots;
    const uint8_t fl = active ? st.flags[b] : 0;
    const int s = active ? st.s[b] : 0;
    if (word < st.W) {
        const uint64_t pw = __ballot((fl & kPred) != 0);
        const uint64_t fw = __ballot((fl & kFail) != 0);
        if (lane == 0) {
            if (st.obs_pred) st.obs_pred[word] = pw;
            if (st.fail) st.fail[word] = fw;
        }
    }
    if (active) {
        if (st.shot_flags) st.shot_flags[b] = fl;
        if (st.shot_s) st.shot_s[b] = s;
    }
    if (st.counters) {
        const bool ovf = (fl & kOverflow) != 0;
        unsigned long long v[6] = {
            active ? 1ull : 0ull,
            (active && (fl & kFail)) ? 1ull : 0ull,
            (active && !ovf && s >= 2 && !(fl & kConvergedAny)) ? 1ull : 0ull,
            (active && (fl & kFcChosen)) ? 1ull : 0ull,
            active ? (unsigned long long)s : 0ull,
            (active && ovf) ? 1ull : 0ull};
        for (int k = 0; k < 6; ++k) {
            unsigned long long x = v[k];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
            if (lane == 0 && x) atomicAdd(&acc[k], x);
        }
        __syncthreads();
        if (tid < 6 && acc[tid]) atomicAdd(&st.counters[tid], acc[tid]);
    }
}

// Copies the instance table of a call into device memory (a kernel rather
// than a host copy, so that the call can be captured into a graph).
struct InstanceTable {
    Instance inst[kMaxInstances];
};

__global__ void k_setup(InstanceTable t, int n, Instance *dst) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&t.inst[0]);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    const int words = (int)(n * sizeof(Instance) / 4);
    for (int i = threadIdx.x; i < words; i += blockDim.x) d[i] = src[i];
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- launches

hipError_t launch_sample(const DevGraph &g, uint64_t seed, uint64_t shot0, uint64_t n, uint64_t *syn,
                         uint64_t *obs, uint64_t *err, hipStream_t stream) {
    const uint64_t W = (n + 63) / 64;
    if (W == 0) return hipSuccess;
    const int nwords = (g.n_det + 31) / 32;
    int bd = 256;
    while (bd > 64 && (size_t)nwords * bd * 4 > 64 * 1024) bd >>= 1;
    const size_t lds = (size_t)nwords * bd * 4;
    const uint64_t grid = (W * 64 + bd - 1) / bd;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)grid), dim3(bd), lds, stream, g, seed, shot0, n, W, nwords, syn,
                       obs, err);
    return hipGetLastError();
}

hipError_t launch_sample_depol(const TannerDev &tn, uint64_t seed, uint64_t shot0, uint64_t n, uint32_t t1,
                               uint32_t t2, uint32_t t3, uint64_t *synx, uint64_t *synz, uint64_t *obs,
                               hipStream_t stream) {
    const uint64_t W = (n + 63) / 64;
    if (W == 0) return hipSuccess;
    const int nwords = (tn.n_xc + tn.n_zc + 31) / 32;
    int bd = 256;
    while (bd > 64 && (size_t)nwords * bd * 4 > 64 * 1024) bd >>= 1;
    if ((size_t)nwords * bd * 4 > 64 * 1024) return hipErrorInvalidValue;
    const size_t lds = (size_t)nwords * bd * 4;
    const uint64_t grid = (W * 64 + bd - 1) / bd;
    hipLaunchKernelGGL(k_sample_depol, dim3((unsigned)grid), dim3(bd), lds, stream, tn, seed, shot0, n, W, nwords,
                       t1, t2, t3, synx, synz, obs);
    return hipGetLastError();
}

hipError_t launch_fill(uint64_t *p, uint64_t n, uint64_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint64_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)grid), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

// Blocks of 256 threads per instance in the per-shot launches.
uint64_t shot_blocks(uint64_t n_shots) { return ((n_shots + 63) / 64 * 64 + 255) / 256; }

hipError_t launch_setup(const Instance *inst, int n, Instance *dst, hipStream_t stream) {
    static_assert(sizeof(Instance) % 4 == 0, "word copy");
    static_assert(sizeof(InstanceTable) <= 4096, "kernel argument size");
    if (n < 1 || n > kMaxInstances) return hipErrorInvalidValue;
    InstanceTable t{};
    for (int i = 0; i < n; ++i) t.inst[i] = inst[i];
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, stream, t, n, dst);
    return hipGetLastError();
}

hipError_t launch_extract(const DecodeShared &c, uint64_t blocks, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3((unsigned)blocks), dim3(256), 0, stream, c);
    return hipGetLastError();
}

hipError_t launch_finalize(const DecodeShared &c, uint64_t blocks, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(256), 0, stream, c);
    return hipGetLastError();
}

}  // namespace bpm
