// gfx950 kernels of the state-vector simulator.
//
// State layout: 2^n interleaved complex amplitudes (complex64 or complex128),
// amplitude index i = sum_q b_q 2^q (Section 3.2).  Batches place states
// `sstride` elements apart.
//
// Operators.  A fused k-qubit operator M (2^k x 2^k) is stored by its XOR-
// shift diagonals: M[r][r ^ m] for the shifts m whose diagonal is nonzero
// (bit m of `present`), so that the group update of Eq. (1q-op)/(2q-op),
// generalised to k qubits, reads
//     y[r] = sum_{m present} d_m[r] * x[r ^ m].
// A dense operator has all 2^k shifts; a Pauli-string exponential has two
// (m = 0 and m = its X/Y mask); diagonal gates one.  The shift loop is
// unrolled at compile time and the test of `present` is wave-uniform, so an
// absent diagonal costs a scalar branch and no vector work.
//
// Reductions (probabilities, norms, Pauli overlaps) accumulate in FP64 with a
// fixed order: per-thread sequential sums, a butterfly within the wave read
// from lane 0, wave partials summed in index order, then chunk partials
// summed in index order by a finishing kernel.  No floating-point atomics, so
// results are bit-identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "launch.h"
#include "swizzle.h"

namespace qk {

using qs::DevOp;

constexpr int NT = 256;            // threads per workgroup (4 waves of 64)
constexpr int NWAVES = NT / 64;

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ void cmac(Cx<T> &acc, const Cx<T> c, const Cx<T> x) {
    acc.re = fma(c.re, x.re, acc.re);
    acc.re = fma(-c.im, x.im, acc.re);
    acc.im = fma(c.re, x.im, acc.im);
    acc.im = fma(c.im, x.re, acc.im);
}

// c * x, rounded exactly as cmac into a zero accumulator
template <typename T>
__device__ __forceinline__ Cx<T> cmul(const Cx<T> c, const Cx<T> x) {
    Cx<T> r;
    r.re = fma(-c.im, x.im, c.re * x.re);
    r.im = fma(c.im, x.re, c.re * x.im);
    return r;
}

#ifndef APPLY_CHUNK_C128
#define APPLY_CHUNK_C128 2
#endif

template <int V>
struct IntC {
    static constexpr int value = V;
};
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(IntC<B>{});
        static_for<B + 1, E>(f);
    }
}

// y[r] = sum over present shifts m of d_m[r] * x[r ^ m]; cf holds the present
// diagonals in ascending m, 2^K entries each.  Outputs R0 .. R0+RC-1 only, so
// that a caller can store one chunk before computing the next and keep fewer
// registers live; every output sums its terms in ascending m.
template <typename T, int K, int R0, int RC>
__device__ __forceinline__ void apply_chunk(const Cx<T> (&x)[1 << K], Cx<T> (&y)[RC],
                                            uint32_t present, const Cx<T> *__restrict__ cf) {
    constexpr int D = 1 << K;
#pragma unroll
    for (int r = 0; r < RC; r++) y[r] = Cx<T>{T(0), T(0)};
    int ti = 0;
#pragma unroll
    for (int m = 0; m < D; m++) {
        if (present & (1u << m)) {
            const Cx<T> *c = cf + ti * D + R0;
#pragma unroll
            for (int r = 0; r < RC; r++) cmac(y[r], c[r], x[(R0 + r) ^ m]);
            ti++;
        }
    }
}

// The same with the coefficients in LDS at byte address cfb (every lane
// reads the same words: broadcast reads, completed in order).
template <typename T, int K, int R0, int RC>
__device__ __forceinline__ void apply_chunk_lds(const Cx<T> (&x)[1 << K], Cx<T> (&y)[RC],
                                                uint32_t present, uint32_t cfb);

template <typename T, int K>
__device__ __forceinline__ void apply_group(const Cx<T> (&x)[1 << K], Cx<T> (&y)[1 << K],
                                            uint32_t present, const Cx<T> *__restrict__ cf) {
    apply_chunk<T, K, 0, (1 << K)>(x, y, present, cf);
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of `v` over the workgroup, identical on every thread, fixed order;
// `red` holds NV * NW doubles of LDS.
template <int NV, int NW, typename P>
__device__ __forceinline__ void block_sum_in(double (&v)[NV], P red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        double s = wave_sum(v[i]);
        if (lane == 0) red[i * NW + w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; i++) {
        double s = 0;
#pragma unroll
        for (int j = 0; j < NW; j++) s += red[i * NW + j];
        v[i] = s;
    }
    __syncthreads();
}

template <int NV, int NW = NWAVES>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NV * NW];
    block_sum_in<NV, NW>(v, &red[0]);
}

template <typename T>
__device__ __forceinline__ double norm2(const Cx<T> a) {
    const double re = double(a.re), im = double(a.im);
    return re * re + im * im;
}

// LDS slot of tile element j (the fold defined with the pass packer).
template <typename T>
__device__ __forceinline__ int sw(int j) {
    return qs::lds_slot(int(sizeof(Cx<T>)), j);
}

// The tile of k_tile sits at LDS byte 0 of its workgroup (the kernel has no
// static LDS, which init_kernels checks), slot i at byte i * sizeof(Cx<T>),
// and is addressed by byte offsets, so that an access costs one XOR; the FP64
// reduction scratch of in-tile measurements follows the tile.
template <typename T>
struct LdsTile {
    static constexpr int LOGE = sizeof(Cx<T>) == 8 ? 3 : 4;
    typedef T V2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ Cx<T> ld(uint32_t byte) {
        const V2 v = *reinterpret_cast<const __attribute__((address_space(3))) V2 *>(uintptr_t(byte));
        return Cx<T>{v.x, v.y};
    }
    static __device__ __forceinline__ void st(uint32_t byte, Cx<T> c) {
        V2 v;
        v.x = c.re;
        v.y = c.im;
        *reinterpret_cast<__attribute__((address_space(3))) V2 *>(uintptr_t(byte)) = v;
    }
    static __device__ __forceinline__ Cx<T> at(int j) { return ld(uint32_t(sw<T>(j)) << LOGE); }
    static __device__ __forceinline__ void set(int j, Cx<T> v) { st(uint32_t(sw<T>(j)) << LOGE, v); }
    static __device__ __forceinline__ __attribute__((address_space(3))) double *red(int t) {
        return reinterpret_cast<__attribute__((address_space(3))) double *>(uintptr_t(uint32_t(sizeof(Cx<T>)) << t));
    }
};

// ------------------------------------------------------------ tile kernel
// Operator record fields, read as eight scalar words (see qs::DevOp).
struct OpRec {
    uint32_t coef, present;
    int k, kind, kx;
    int pos[5];
    int slot[5];
    int xq[5];
};

// The record at LDS byte address `at` (the same for every lane): eight words,
// moved to scalar registers.
__device__ __forceinline__ OpRec decode_op(uint32_t at) {
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const U4 a = *reinterpret_cast<const __attribute__((address_space(3))) U4 *>(uintptr_t(at));
    const U4 bq = *reinterpret_cast<const __attribute__((address_space(3))) U4 *>(uintptr_t(at + 16));
    uint32_t w[8] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w};
#pragma unroll
    for (int i = 0; i < 8; i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    OpRec o;
    o.coef = w[0];
    o.present = w[1];
    o.k = int(w[2] & 0xff);
    o.pos[0] = int((w[2] >> 8) & 0xff);
    o.pos[1] = int((w[2] >> 16) & 0xff);
    o.pos[2] = int(w[2] >> 24);
    o.pos[3] = int(w[3] & 0xff);
    o.pos[4] = int((w[3] >> 8) & 0xff);
    o.kind = int((w[3] >> 16) & 0xff);
    o.kx = int(w[3] >> 24);
    o.slot[0] = int(w[4] & 0xffff);
    o.slot[1] = int(w[4] >> 16);
    o.slot[2] = int(w[5] & 0xffff);
    o.slot[3] = int(w[5] >> 16);
    o.slot[4] = int(w[6] & 0xffff);
    o.xq[0] = int((w[6] >> 16) & 0xff);
    o.xq[1] = int(w[6] >> 24);
    o.xq[2] = int(w[7] & 0xff);
    o.xq[3] = int((w[7] >> 8) & 0xff);
    o.xq[4] = int((w[7] >> 16) & 0xff);
    return o;
}

template <typename T, int K, int R0, int RC>
__device__ __forceinline__ void apply_chunk_lds(const Cx<T> (&x)[1 << K], Cx<T> (&y)[RC],
                                                uint32_t present, uint32_t cfb) {
    using L = LdsTile<T>;
    constexpr int D = 1 << K;
    uint32_t c = cfb + (uint32_t(R0) << L::LOGE);
    // A shift's RC coefficients are all read before its first multiply-add
    // (the scheduling barrier keeps the reads together), so that one LDS
    // latency covers them.
    Cx<T> cv[RC];
    // the main diagonal (present in most operators) starts the sums
    if (present & 1u) {
#pragma unroll
        for (int r = 0; r < RC; r++) cv[r] = L::ld(c + (uint32_t(r) << L::LOGE));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < RC; r++) y[r] = cmul(cv[r], x[R0 + r]);
        c += uint32_t(D) << L::LOGE;
    } else {
#pragma unroll
        for (int r = 0; r < RC; r++) y[r] = Cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int m = 1; m < D; m++) {
        if (present & (1u << m)) {
#pragma unroll
            for (int r = 0; r < RC; r++) cv[r] = L::ld(c + (uint32_t(r) << L::LOGE));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < RC; r++) cmac(y[r], cv[r], x[(R0 + r) ^ m]);
            c += uint32_t(D) << L::LOGE;
        }
    }
}

// y[i][r] = sum over present shifts m of d_m[r] * x[i][r ^ m] for NB groups
// that share the operator: each coefficient is read from LDS once (a
// broadcast read) and applied to every group, in ascending m as above.
template <typename T, int K, int NB>
__device__ __forceinline__ void apply_groups_lds(const Cx<T> (&x)[NB][1 << K], Cx<T> (&y)[NB][1 << K],
                                                 uint32_t present, uint32_t cfb) {
    using L = LdsTile<T>;
    constexpr int D = 1 << K;
    uint32_t c = cfb;
    Cx<T> cv[D];
    if (present & 1u) {
#pragma unroll
        for (int r = 0; r < D; r++) cv[r] = L::ld(c + (uint32_t(r) << L::LOGE));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < D; r++)
#pragma unroll
            for (int i = 0; i < NB; i++) y[i][r] = cmul(cv[r], x[i][r]);
        c += uint32_t(D) << L::LOGE;
    } else {
#pragma unroll
        for (int i = 0; i < NB; i++)
#pragma unroll
            for (int r = 0; r < D; r++) y[i][r] = Cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int m = 1; m < D; m++) {
        if (present & (1u << m)) {
#pragma unroll
            for (int r = 0; r < D; r++) cv[r] = L::ld(c + (uint32_t(r) << L::LOGE));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < D; r++)
#pragma unroll
                for (int i = 0; i < NB; i++) cmac(y[i][r], cv[r], x[i][r ^ m]);
            c += uint32_t(D) << L::LOGE;
        }
    }
}

// Byte addresses of the members of a thread's first group (g = threadIdx.x)
// for an operator of at most 4 qubits: they depend on its record only, so they
// are computed before the barrier that ends the previous operator.  Entries
// beyond 2^k are unused.
template <typename T>
__device__ __forceinline__ void prep_addr(const OpRec &op, uint32_t (&addr)[16]) {
    using L = LdsTile<T>;
    int base = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (j < op.k) base = ((base >> op.pos[j]) << (op.pos[j] + 1)) | (base & ((1 << op.pos[j]) - 1));
    const uint32_t b0 = uint32_t(sw<T>(base)) << L::LOGE;
    // (the fold is linear: slot(base | off) = slot(base) ^ slot(off); slots
    // beyond the operator's k are zero in the record)
    uint32_t off[16];
    off[0] = 0;
#pragma unroll
    for (int r = 1; r < 16; r++) off[r] = off[r & (r - 1)] ^ (uint32_t(op.slot[__builtin_ctz(r)]) << L::LOGE);
#pragma unroll
    for (int r = 0; r < 16; r++) {
        addr[r] = b0 ^ off[r];
        // keep the addresses in registers across the barrier and for the
        // write-back
        asm volatile("" : "+v"(addr[r]));
    }
}

// One operator on the tile in LDS.  The tile has 2^t = E * TNT elements
// (E = 2^LE per thread when t > log2 TNT) in 2^(t-K) groups of 2^K.  With
// K >= LE a thread has at most one group, at addr0.  With K < LE it has
// 2^(LE-K) groups, tid + i * TNT for i < 2^(LE-K); inserting the operator's
// zero bits and the LDS fold are both linear, so group i's members sit at
// addr0[r] ^ gof(i), where gof is the same on every lane.  Up to 16 of a
// thread's amplitudes are loaded before the first multiply, so that the LDS
// latency is paid once per batch rather than once per group.
template <typename T, int K, int LE, int TNT>
__device__ __forceinline__ void apply_lds(int t, const OpRec &op, uint32_t cfb, const uint32_t (&addr0)[16]) {
    using L = LdsTile<T>;
    constexpr int D = 1 << K;
    // complex128 computes and stores the outputs in chunks of RC when 512
    // threads share the CU, to keep 4 waves per SIMD
    constexpr int RC = (sizeof(T) == 8 && TNT == 512 && D > APPLY_CHUNK_C128) ? APPLY_CHUNK_C128 : D;
    auto compute_store = [&](const Cx<T> (&x)[D], uint32_t gofs) {
        static_for<0, D / RC>([&](auto ci) {
            constexpr int R0 = decltype(ci)::value * RC;
            Cx<T> y[RC];
            apply_chunk_lds<T, K, R0, RC>(x, y, op.present, cfb);
#pragma unroll
            for (int r = 0; r < RC; r++) L::st(addr0[R0 + r] ^ gofs, y[r]);
        });
    };
    if constexpr (K >= LE) {
        if (int(threadIdx.x) < (1 << (t - K))) {
            Cx<T> x[D];
#pragma unroll
            for (int r = 0; r < D; r++) x[r] = L::ld(addr0[r]);
            compute_store(x, 0u);
        }
    } else {
        constexpr int LOGT = (TNT == 512) ? 9 : 8;
        constexpr int LG = LE - K;                                  // log2 groups per thread
        // log2 amplitudes per batch: 16, or 32 for whole 14-qubit complex64
        // states (one workgroup per CU, so registers are plentiful)
        constexpr int MB = (sizeof(T) == 4 && LE == 5 && TNT == 512) ? 5 : 4;
        constexpr int LB = (LG < MB - K) ? LG : (K >= MB ? 0 : MB - K);   // log2 groups per batch
        // offsets of the basis groups 2^b * TNT
        uint32_t gb[LG];
#pragma unroll
        for (int b = 0; b < LG; b++) {
            int x = 1 << (LOGT + b);
#pragma unroll
            for (int j = 0; j < K; j++) x = ((x >> op.pos[j]) << (op.pos[j] + 1)) | (x & ((1 << op.pos[j]) - 1));
            gb[b] = uint32_t(sw<T>(x)) << L::LOGE;
        }
        for (int bi = 0; bi < (1 << (LG - LB)); bi++) {
            uint32_t g0 = 0;
#pragma unroll
            for (int b = 0; b < LG - LB; b++)
                if ((bi >> b) & 1) g0 ^= gb[LB + b];
            uint32_t gofs[1 << LB];
            Cx<T> x[1 << LB][D];
#pragma unroll
            for (int i = 0; i < (1 << LB); i++) {
                uint32_t o = g0;
#pragma unroll
                for (int b = 0; b < LB; b++)
                    if ((i >> b) & 1) o ^= gb[b];
                gofs[i] = o;
#pragma unroll
                for (int r = 0; r < D; r++) x[i][r] = L::ld(addr0[r] ^ o);
            }
            Cx<T> y[1 << LB][D];
            apply_groups_lds<T, K, (1 << LB)>(x, y, op.present, cfb);
#pragma unroll
            for (int i = 0; i < (1 << LB); i++)
#pragma unroll
                for (int r = 0; r < D; r++) L::st(addr0[r] ^ gofs[i], y[i][r]);
        }
    }
}

// An operator applied to a thread's registers: element tid + i * TNT sits at
// tile position log2(TNT) + b for bit b of the register index i, so an
// operator whose tile positions are log2(TNT) + OFF + j has the groups
// i = hi * 2^(OFF+K) + r * 2^OFF + lo (members r).  The first operator of a
// pass runs so on the tile as loaded, the last one on the tile as it leaves
// LDS for the store.  Coefficients are read through uniform addresses; the
// sums follow the same order as in LDS (main diagonal first, then ascending
// shifts).
template <typename T, int K, int OFF, int LE>
__device__ __forceinline__ void regs_apply(Cx<T> (&v)[1 << LE], uint32_t present, const Cx<T> *__restrict__ c) {
    if constexpr (K + OFF <= LE) {
        constexpr int D = 1 << K;
#pragma unroll
        for (int hi = 0; hi < (1 << (LE - OFF - K)); hi++) {
#pragma unroll
            for (int lo = 0; lo < (1 << OFF); lo++) {
                Cx<T> x[D], y[D];
#pragma unroll
                for (int r = 0; r < D; r++) x[r] = v[(hi << (OFF + K)) | (r << OFF) | lo];
                uint32_t t0 = 0;
                if (present & 1u) {
#pragma unroll
                    for (int r = 0; r < D; r++) y[r] = cmul(c[r], x[r]);
                    t0 = D;
                } else {
#pragma unroll
                    for (int r = 0; r < D; r++) y[r] = Cx<T>{T(0), T(0)};
                }
#pragma unroll
                for (int m = 1; m < D; m++) {
                    if (present & (1u << m)) {
#pragma unroll
                        for (int r = 0; r < D; r++) cmac(y[r], c[t0 + r], x[r ^ m]);
                        t0 += D;
                    }
                }
#pragma unroll
                for (int r = 0; r < D; r++) v[(hi << (OFF + K)) | (r << OFF) | lo] = y[r];
            }
        }
    }
}

// Widest operator run on the registers (the host's first_regs_max_k): the
// host places only operators of at most this many tile qubits there.
template <typename T>
constexpr int first_regs_max_k() { return 4; }

template <typename T, int OFF, int LE>
__device__ __forceinline__ void regs_apply_k(Cx<T> (&v)[1 << LE], int k, uint32_t present,
                                             const Cx<T> *__restrict__ c) {
    constexpr int MK = first_regs_max_k<T>();
    switch (k) {
    case 0: regs_apply<T, 0, OFF, LE>(v, present, c); break;
    case 1: regs_apply<T, 1, OFF, LE>(v, present, c); break;
    case 2: regs_apply<T, 2, OFF, LE>(v, present, c); break;
    case 3: if constexpr (MK >= 3) regs_apply<T, 3, OFF, LE>(v, present, c); break;
    default: if constexpr (MK >= 4) regs_apply<T, 4, OFF, LE>(v, present, c); break;
    }
}

// The record at `rec` (global memory) applied to the registers, its tile
// positions starting at register-index bit `off`.
template <typename T, int LE>
__device__ __forceinline__ void regs_record(Cx<T> (&v)[1 << LE], const DevOp *__restrict__ rec,
                                            const Cx<T> *__restrict__ cfs, uint64_t base, int off) {
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const U4 a = reinterpret_cast<const U4 *>(rec)[0];
    const U4 bq = reinterpret_cast<const U4 *>(rec)[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w};
    uint32_t u[8];
#pragma unroll
    for (int x = 0; x < 8; x++) u[x] = __builtin_amdgcn_readfirstlane(w[x]);
    const uint32_t present = u[1];
    const int k = int(u[2] & 0xff);
    const int kx = int(u[3] >> 24);
    const int xq[5] = {int((u[6] >> 16) & 0xff), int(u[6] >> 24), int(u[7] & 0xff), int((u[7] >> 8) & 0xff),
                       int((u[7] >> 16) & 0xff)};
    uint32_t cf = u[0];
    // block qubits outside the tile select the coefficient block (constant
    // indices keep the fields in registers)
    uint32_t e = 0;
#pragma unroll
    for (int j = 0; j < 5; j++)
        if (j < kx) e |= uint32_t((base >> xq[j]) & 1) << j;
    cf += (e * uint32_t(__builtin_popcount(present))) << k;
    const Cx<T> *c = cfs + cf;
    switch (off) {
    case 0: regs_apply_k<T, 0, LE>(v, k, present, c); break;
    case 1: regs_apply_k<T, 1, LE>(v, k, present, c); break;
    case 2: regs_apply_k<T, 2, LE>(v, k, present, c); break;
    default: regs_apply_k<T, 3, LE>(v, k, present, c); break;
    }
}

// Scatter the low bits of x into the set bits of m, in ascending order.
__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t m) {
    uint64_t r = 0;
    while (m && x) {
        const uint64_t lo = m & (~m + 1);
        if (x & 1) r |= lo;
        x >>= 1;
        m &= m - 1;
    }
    return r;
}

// Measurement, assertion, reset, and measurement then reset, inside a
// resident program (t == n, so the LDS index is the amplitude index).
// Returns 0 or a negative status.  Thread tid holds the elements j = tid + i * TNT (i < E; with E = 1 and
// t < log2 TNT only the first 2^t threads); the fold is linear, so element j
// sits at slot sw(tid) ^ sw(i * TNT), with sw(i * TNT) the XOR of the
// constants sw(TNT << c) over the set bits c of i, and its partner j ^ 2^q at
// that slot ^ sw(2^q).  The sums over j run in ascending i on every thread,
// then over the threads in fixed order.  The loops stay rolled except for
// whole 14-qubit complex64 states: this code is compiled into every tile
// kernel, whose registers it must not raise.
template <typename T, int LE, int TNT>
__device__ int lds_measure(int t, const OpRec &op, const MeasArgs &ma, uint32_t b) {
    using L = LdsTile<T>;
    constexpr int E = 1 << LE;
    constexpr int LOGT = (TNT == 512) ? 9 : 8;
    // unrolled only where one workgroup fills a CU (whole 14-qubit complex64
    // states) and registers are plentiful
    constexpr int UNR = (LE >= 5) ? E : 1;
    const int q = op.pos[0];
    const int slot = int(op.coef);
    const int tid = threadIdx.x;
    const bool active = (E > 1) || (tid < (1 << t));
    const uint32_t stid = uint32_t(sw<T>(tid)) << L::LOGE;
    auto addr = [&](int i) {
        uint32_t a = stid;
#pragma unroll
        for (int c = 0; c < LE; c++)
            if ((i >> c) & 1) a ^= uint32_t(sw<T>(TNT << c)) << L::LOGE;
        return a;
    };
    auto bit = [&](int i) { return q < LOGT ? (tid >> q) & 1 : (i >> (q - LOGT)) & 1; };
    double w[2] = {0.0, 0.0};
#pragma unroll UNR
    for (int i = 0; i < E; i++)
        if (active) w[bit(i)] += norm2(L::ld(addr(i)));
    block_sum_in<2, TNT / 64>(w, L::red(t));
    const double P0 = w[0], P1 = w[1];
    // Each pair (j, j | 2^q) rewritten by the thread that holds j: j takes
    // s times the amplitude at j ^ src, j | 2^q becomes 0.
    const uint32_t dq = uint32_t(sw<T>(1 << q)) << L::LOGE;
    auto to_zero = [&](uint32_t src, T s) {
#pragma unroll UNR
        for (int i = 0; i < E; i++) {
            if (active && bit(i) == 0) {
                const uint32_t a = addr(i);
                Cx<T> c = L::ld(a ^ src);
                c.re *= s;
                c.im *= s;
                L::st(a, c);
                L::st(a ^ dq, Cx<T>{T(0), T(0)});
            }
        }
    };
    if (op.kind == qs::DEVOP_RESET) {
        if (P1 == 0.0) return 0;
        if (P0 != 0.0) return QSIM_E_NOT_DEFINITE;
        to_zero(dq, T(1));
        return 0;
    }
    int o;
    const size_t idx = size_t(b) * ma.nslots + slot;
    if (op.kind == qs::DEVOP_ASSERT0) {
        if (!(P0 > 0.0)) return QSIM_E_ZERO_PROB;
        o = 0;
    } else if (ma.forced && ma.forced[idx] >= 0) {
        o = ma.forced[idx];
        if (!((o ? P1 : P0) > 0.0)) return QSIM_E_ZERO_PROB;
    } else {
        const double p0 = P0 / (P0 + P1);
        o = (ma.uniforms[idx] < p0) ? 0 : 1;
    }
    const double kept = o ? P1 : P0;
    const T scale = T(1.0 / sqrt(kept));
    if (threadIdx.x == 0) {
        ma.outcomes[idx] = o;
        ma.probs[idx] = kept / (P0 + P1);
    }
    if (op.kind == qs::DEVOP_MEASURE_RESET) {
        // collapse onto outcome o and move it to |0> in one rewrite
        to_zero(o ? dq : 0u, scale);
        return 0;
    }
#pragma unroll UNR
    for (int i = 0; i < E; i++) {
        if (active) {
            Cx<T> a = L::ld(addr(i));
            if (bit(i) == o) { a.re *= scale; a.im *= scale; }
            else a = Cx<T>{T(0), T(0)};
            L::st(addr(i), a);
        }
    }
    return 0;
}

// Tile loads and stores of the state stream past the caches (non-temporal):
// each pass touches every amplitude once, and the operator records and
// coefficients read through the scalar cache then stay resident in L2.
template <typename T>
__device__ __forceinline__ Cx<T> ld_stream(const Cx<T> *p) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(p));
    return Cx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_stream(Cx<T> *p, Cx<T> c) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    V2 v;
    v.x = c.re;
    v.y = c.im;
    __builtin_nontemporal_store(v, reinterpret_cast<V2 *>(p));
}

// One tile of 2^t amplitudes per workgroup of TNT threads (blockIdx.x:
// tile, blockIdx.y: state of a batch).  Element j of the tile
// (j = tid + i * TNT, E = 2^LE elements per thread) lives at amplitude
// base | deposit(j, tile_mask),
// where base deposits the tile index into the other qubits.
//
// The pass's operator records [ob, oe) and coefficients [cb, ce) are copied
// into LDS behind the tile while the tile loads are in flight; an operator
// then reads its record and coefficients as LDS broadcasts, which complete in
// order and let its first multiply-adds start as soon as their own
// coefficients arrive.
template <typename T, int LE, int TNT>
__global__ void __launch_bounds__(TNT) k_tile(Cx<T> *__restrict__ state, uint64_t sstride,
                                             TileArgs ta, const DevOp *__restrict__ ops,
                                             uint32_t ob, uint32_t oe,
                                             const Cx<T> *__restrict__ coefs, uint32_t cb,
                                             uint32_t ce, uint64_t cstride, MeasArgs ma,
                                             uint32_t flags) {
    using L = LdsTile<T>;
    constexpr int E = 1 << LE;
    const uint32_t b = blockIdx.y;
    Cx<T> *st = state + size_t(b) * sstride;
    const Cx<T> *cfs = coefs + size_t(b) * cstride;
    const int tid = threadIdx.x;
    const bool active = (E > 1) || (tid < (1 << ta.t));
    if (ma.status && ma.status[b] != 0) return;   // an earlier step of this state failed

    const int nrec = int(oe - ob), ncf = int(ce - cb);
    // LDS: the tile, the reduction scratch, the pass's records, its coefficients
    const uint32_t rec_at = (uint32_t(sizeof(Cx<T>)) << ta.t) + uint32_t(kTileRedBytes);
    const uint32_t cf_at = rec_at + uint32_t(nrec) * uint32_t(sizeof(DevOp));
    const uint64_t base = tile_base(blockIdx.x, ta.rest_mask, ta.nxcd, ta.xcd_q);
    // thread part: the low log2(TNT) bits of j; iteration part: the bits above
    // (tile position j is qubit ta.tq[j])
    constexpr int LOGT = (TNT == 512) ? 9 : 8;
    uint64_t toff = 0;
#pragma unroll
    for (int bt = 0; bt < LOGT; bt++)
        if (bt < ta.t && ((tid >> bt) & 1)) toff |= uint64_t(1) << ta.tq[bt];
    uint64_t ibit[LE > 0 ? LE : 1];
#pragma unroll
    for (int bt = 0; bt < LE; bt++) ibit[bt] = uint64_t(1) << ta.tq[LOGT + bt];

    // element tid + i * TNT sits at slot sw(tid) ^ sw(i * TNT)
    const uint32_t stid = uint32_t(sw<T>(tid)) << L::LOGE;
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const U4 *gops = reinterpret_cast<const U4 *>(ops + ob);
    const Cx<T> *gcf = cfs + cb;
    // The first operator, when placed on the register-index bits, runs on the
    // loaded tile values before they reach LDS (compiled for 2 to 16 elements
    // per thread; LE >= 1 means every thread holds E elements).  A tile that
    // starts as |0...0> leaves it to the operator loop.
    const bool first_regs =
        (LE >= 1 && LE <= 4) && (ta.regs & 1) && nrec > 0 && !(flags & TF_INIT_ZERO);
    // likewise the last operator, on the tile as it leaves LDS for the store
    const bool last_regs = (LE >= 1 && LE <= 4) && (ta.regs & 2) && nrec > (first_regs ? 1 : 0) &&
                           !(flags & TF_NO_STORE);
    const int iend = last_regs ? nrec - 1 : nrec;
    if (flags & TF_INIT_ZERO) {
#pragma unroll
        for (int i = 0; i < E; i++)
            if (active)
                L::st(stid ^ (uint32_t(sw<T>(i * TNT)) << L::LOGE),
                      Cx<T>{T((base == 0 && tid == 0 && i == 0) ? 1 : 0), T(0)});
        for (int x = tid; x < 2 * nrec; x += TNT)
            *reinterpret_cast<__attribute__((address_space(3))) U4 *>(uintptr_t(rec_at + 16u * x)) = gops[x];
        for (int x = tid; x < ncf; x += TNT) L::st(cf_at + (uint32_t(x) << L::LOGE), gcf[x]);
    } else {
        // all E tile loads are in flight before the first LDS write
        Cx<T> v[E];
#pragma unroll
        for (int i = 0; i < E; i++) {
            uint64_t io = 0;
#pragma unroll
            for (int bt = 0; bt < LE; bt++)
                if ((i >> bt) & 1) io |= ibit[bt];
            if (active) v[i] = ld_stream(st + (base | toff | io));
        }
        // the pass's records and coefficients follow while the tile loads fly
        for (int x = tid; x < 2 * nrec; x += TNT)
            *reinterpret_cast<__attribute__((address_space(3))) U4 *>(uintptr_t(rec_at + 16u * x)) = gops[x];
        for (int x = tid; x < ncf; x += TNT) L::st(cf_at + (uint32_t(x) << L::LOGE), gcf[x]);
        if constexpr (LE >= 1 && LE <= 4) {
            if (first_regs) regs_record<T, LE>(v, ops + ob, cfs, base, 0);
        }
#pragma unroll
        for (int i = 0; i < E; i++)
            if (active) L::st(stid ^ (uint32_t(sw<T>(i * TNT)) << L::LOGE), v[i]);
    }
    __syncthreads();

    int status = 0;
    int i = first_regs ? 1 : 0;
    // the next operator's record and addresses are prepared before the
    // barrier that ends the current one
    OpRec op{};
    uint32_t addr[16];
    if (i < iend) {
        op = decode_op(rec_at + uint32_t(i) * uint32_t(sizeof(DevOp)));
        if (op.kind == qs::DEVOP_MAT) prep_addr<T>(op, addr);
    }
    for (; i < iend; i++) {
        if (op.kind == qs::DEVOP_MAT) {
            uint32_t cf = op.coef - cb;
            if (op.kx) {
                // the qubits the operator is diagonal on that lie outside the
                // tile are fixed for the whole tile: they pick the block of
                // coefficients (popcount(present) << k entries each)
                // (constant indices keep the record's fields in registers)
                uint32_t e = 0;
#pragma unroll
                for (int j = 0; j < 5; j++)
                    if (j < op.kx) e |= uint32_t((base >> op.xq[j]) & 1) << j;
                cf += (e * uint32_t(__builtin_popcount(op.present))) << op.k;
            }
            cf = cf_at + (cf << L::LOGE);
            // operators addressing up to 4 tile qubits (wider ones run as
            // strided sweeps, which keeps the kernel's registers low enough
            // for the occupancy the tile's LDS allows)
            switch (op.k) {
            case 0: apply_lds<T, 0, LE, TNT>(ta.t, op, cf, addr); break;
            case 1: apply_lds<T, 1, LE, TNT>(ta.t, op, cf, addr); break;
            case 2: apply_lds<T, 2, LE, TNT>(ta.t, op, cf, addr); break;
            case 3: apply_lds<T, 3, LE, TNT>(ta.t, op, cf, addr); break;
            default: apply_lds<T, 4, LE, TNT>(ta.t, op, cf, addr); break;
            }
        } else {
            // the same on every lane: keeps the loop (and the record
            // addresses) uniform
            status = __builtin_amdgcn_readfirstlane(lds_measure<T, LE, TNT>(ta.t, op, ma, b));
        }
        if (i + 1 < iend) {
            op = decode_op(rec_at + uint32_t(i + 1) * uint32_t(sizeof(DevOp)));
            if (op.kind == qs::DEVOP_MAT) prep_addr<T>(op, addr);
        }
        __syncthreads();
        if (status) break;
    }
    if (status && ma.status && tid == 0) {
        ma.status[b] = status;
        if (ma.fail_at) ma.fail_at[b] = int(ob) + i;
    }
    if (!(flags & TF_NO_STORE)) {
        Cx<T> w[E];
#pragma unroll
        for (int i2 = 0; i2 < E; i2++)
            if (active) w[i2] = L::ld(stid ^ (uint32_t(sw<T>(i2 * TNT)) << L::LOGE));
        if constexpr (LE >= 1 && LE <= 4) {
            if (last_regs && !status) regs_record<T, LE>(w, ops + ob + (nrec - 1), cfs, base, (ta.regs >> 2) & 7);
        }
#pragma unroll
        for (int i2 = 0; i2 < E; i2++) {
            uint64_t io = 0;
#pragma unroll
            for (int bt = 0; bt < LE; bt++)
                if ((i2 >> bt) & 1) io |= ibit[bt];
            if (active) st_stream(st + (base | toff | io), w[i2]);
        }
    }
}

// ------------------------------------------------ register-resident pass
// Thread `tid` of a 2^LOGT-thread workgroup holds 16 amplitudes of the tile
// in v[0..15]; element (tid, i) sits at position bits tid (lane bits 0..5,
// wave bits 6..LOGT-1) and i (register bits LOGT..LOGT+3).  A layout names
// the canonical tile bit each position carries (see the host planner).

// Exchange lane bit 5 (LANE5) or 4 with register bit RB: registers i and
// i | 2^RB trade the half of their lanes whose lane bit differs from the
// register bit (v_permlane32_swap / v_permlane16_swap on every 32-bit word).
template <typename T, int RB, bool LANE5>
__device__ __forceinline__ void reg_swap(Cx<T> (&v)[16]) {
    constexpr int W = int(sizeof(Cx<T>) / 4);
    static_for<0, 16>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (!((i >> RB) & 1)) {
            constexpr int j = i | (1 << RB);
            uint32_t a[W], b[W];
            __builtin_memcpy(a, &v[i], sizeof(a));
            __builtin_memcpy(b, &v[j], sizeof(b));
#pragma unroll
            for (int d = 0; d < W; d++) {
                if constexpr (LANE5) {
                    const auto r = __builtin_amdgcn_permlane32_swap(a[d], b[d], false, false);
                    a[d] = r[0];
                    b[d] = r[1];
                } else {
                    const auto r = __builtin_amdgcn_permlane16_swap(a[d], b[d], false, false);
                    a[d] = r[0];
                    b[d] = r[1];
                }
            }
            __builtin_memcpy(&v[i], a, sizeof(a));
            __builtin_memcpy(&v[j], b, sizeof(b));
        }
    });
}

template <typename T, bool LANE5>
__device__ __forceinline__ void reg_swap_rb(Cx<T> (&v)[16], int rb) {
    switch (rb) {
    case 0: reg_swap<T, 0, LANE5>(v); break;
    case 1: reg_swap<T, 1, LANE5>(v); break;
    case 2: reg_swap<T, 2, LANE5>(v); break;
    default: reg_swap<T, 3, LANE5>(v); break;
    }
}

// An operator on the 4 register bits: y[r] = sum over present register
// shifts M (main diagonal first, then ascending) of c_M[r] * v[r ^ M], with
// the 16 coefficients of each present shift at c (uniform addresses: scalar
// loads).  Every thread applies it to its own registers.
template <typename T>
__device__ __forceinline__ void reg_apply(Cx<T> (&v)[16], uint32_t present, const Cx<T> *__restrict__ c) {
    Cx<T> y[16];
    uint32_t t0 = 0;
    if (present & 1u) {
#pragma unroll
        for (int r = 0; r < 16; r++) y[r] = cmul(c[r], v[r]);
        t0 = 16;
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) y[r] = Cx<T>{T(0), T(0)};
    }
    static_for<1, 16>([&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if (present & (1u << M)) {
#pragma unroll
            for (int r = 0; r < 16; r++) cmac(y[r], c[t0 + r], v[r ^ M]);
            t0 += 16;
        }
    });
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = y[r];
}

// The LDS byte address of every element of a thread under layout `pos`
// (canonical bit per position): the tile's canonical index j sits at slot
// sw(j), and the fold is linear, so the thread part and the register part
// combine by XOR.
template <typename T, int LOGT>
__device__ __forceinline__ void reg_lds_addr(const uint8_t (&pos)[16], uint32_t (&addr)[16]) {
    using L = LdsTile<T>;
    const int tid = threadIdx.x;
    int tj = 0;
#pragma unroll
    for (int bt = 0; bt < LOGT; bt++)
        if ((tid >> bt) & 1) tj |= 1 << pos[bt];
    const uint32_t stp = uint32_t(sw<T>(tj)) << L::LOGE;
    uint32_t sib[4];
#pragma unroll
    for (int b = 0; b < 4; b++) sib[b] = uint32_t(sw<T>(1 << pos[LOGT + b])) << L::LOGE;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        uint32_t a = stp;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if ((i >> b) & 1) a ^= sib[b];
        addr[i] = a;
    }
}

// The eight words of the record at LDS byte address `at`, in scalar
// registers (every lane reads the same words).
__device__ __forceinline__ void reg_rec(uint32_t at, uint32_t (&w)[8]) {
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const U4 a = *reinterpret_cast<const __attribute__((address_space(3))) U4 *>(uintptr_t(at));
    const U4 b = *reinterpret_cast<const __attribute__((address_space(3))) U4 *>(uintptr_t(at + 16));
    const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 8; i++) w[i] = __builtin_amdgcn_readfirstlane(x[i]);
}

__device__ __forceinline__ void rec_bytes(const uint32_t (&w)[8], uint8_t (&pos)[16]) {
#pragma unroll
    for (int x = 0; x < 16; x++) pos[x] = uint8_t((w[x >> 2] >> (8 * (x & 3))) & 0xff);
}

// LDS of a register-resident pass: the tile (only for passes with
// re-layouts), then the pass's records, copied at the start so that a
// record costs an LDS read instead of a trip to memory.
template <typename T, int LOGT>
__global__ void __launch_bounds__(1 << LOGT) k_reg(Cx<T> *__restrict__ state, uint64_t sstride, RegArgs ra,
                                                  const DevOp *__restrict__ ops, uint32_t ob, uint32_t oe,
                                                  const Cx<T> *__restrict__ coefs, uint32_t cb, uint32_t ce,
                                                  uint64_t cstride, const int32_t *__restrict__ status,
                                                  uint32_t flags) {
    using L = LdsTile<T>;
    constexpr int TNT = 1 << LOGT;
    const uint32_t b = blockIdx.y;
    if (status && status[b] != 0) return;
    Cx<T> *st = state + size_t(b) * sstride;
    const Cx<T> *cfs = coefs + size_t(b) * cstride;
    const int tid = threadIdx.x;
    const uint64_t base = tile_base(blockIdx.x, ra.rest_mask, ra.nxcd, ra.xcd_q);
    const bool nt = (ra.flags & RF_NONTEMPORAL) != 0;
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const uint32_t nrec = oe - ob;
    const uint32_t rec_at = ra.lds_bytes - nrec * uint32_t(sizeof(DevOp));
    // The pass's records: in flight first.  Its coefficients, read later
    // through the scalar cache, are touched once here (one load per 64-byte
    // line, spread over the workgroup) so that those reads find them in L2.
    const U4 *gops = reinterpret_cast<const U4 *>(ops + ob);
    U4 rv[2];
#pragma unroll
    for (int x = 0; x < 2; x++) {
        const uint32_t idx = uint32_t(tid) + uint32_t(x) * TNT;
        if (idx < 2 * nrec) rv[x] = gops[idx];
    }
    {
        const char *c0 = reinterpret_cast<const char *>(cfs + cb);
        const uint32_t lines = ((ce - cb) * uint32_t(sizeof(Cx<T>)) + 63) / 64;
        for (uint32_t x = tid; x < lines; x += TNT) (void)*reinterpret_cast<const volatile uint32_t *>(c0 + 64 * size_t(x));
    }
    // global offsets of a thread's elements in the load layout
    Cx<T> v[16];
    {
        uint64_t toff = 0;
#pragma unroll
        for (int bt = 0; bt < LOGT; bt++)
            if ((tid >> bt) & 1) toff |= uint64_t(1) << ra.tq[ra.load_pos[bt]];
        uint64_t ib[4];
#pragma unroll
        for (int x = 0; x < 4; x++) ib[x] = uint64_t(1) << ra.tq[ra.load_pos[LOGT + x]];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            uint64_t a = base | toff;
#pragma unroll
            for (int x = 0; x < 4; x++)
                if ((i >> x) & 1) a |= ib[x];
            if (flags & TF_INIT_ZERO) v[i] = Cx<T>{T(a == 0 ? 1 : 0), T(0)};
            else v[i] = nt ? ld_stream(st + a) : st[a];
        }
    }
#pragma unroll
    for (int x = 0; x < 2; x++) {
        const uint32_t idx = uint32_t(tid) + uint32_t(x) * TNT;
        if (idx < 2 * nrec)
            *reinterpret_cast<__attribute__((address_space(3))) U4 *>(uintptr_t(rec_at + 16u * idx)) = rv[x];
    }
    for (uint32_t idx = uint32_t(tid) + 2u * TNT; idx < 2 * nrec; idx += TNT)
        *reinterpret_cast<__attribute__((address_space(3))) U4 *>(uintptr_t(rec_at + 16u * idx)) = gops[idx];
    __syncthreads();
    bool xposed = false;
    for (uint32_t at = 0; at < nrec; at++) {
        uint32_t w[8];
        reg_rec(rec_at + at * uint32_t(sizeof(DevOp)), w);
        const int kind = int((w[3] >> 16) & 0xff);
        if (kind == qs::DEVOP_RMAT) {
            uint32_t cf = w[0];
            const uint32_t present = w[1];
            const int kx = int(w[3] >> 24);
            if (kx) {
                // block qubits outside the tile select the coefficient block
                const int xq[5] = {int((w[6] >> 16) & 0xff), int(w[6] >> 24), int(w[7] & 0xff),
                                   int((w[7] >> 8) & 0xff), int((w[7] >> 16) & 0xff)};
                uint32_t e = 0;
#pragma unroll
                for (int j = 0; j < 5; j++)
                    if (j < kx) e |= uint32_t((base >> xq[j]) & 1) << j;
                cf += (e * uint32_t(__builtin_popcount(present))) << 4;
            }
            reg_apply<T>(v, present, cfs + cf);
        } else if (kind == qs::DEVOP_SWAP) {
            const int lane = int((w[2] >> 8) & 0xff), rb = int((w[2] >> 16) & 0xff);
            if (lane == 5) reg_swap_rb<T, true>(v, rb);
            else reg_swap_rb<T, false>(v, rb);
        } else if (kind == qs::DEVOP_XPOSE) {
            // the tile through LDS: written in the layout of this record,
            // read back in the layout of the next one
            uint8_t from[16], to[16];
            rec_bytes(w, from);
            reg_rec(rec_at + (at + 1) * uint32_t(sizeof(DevOp)), w);
            rec_bytes(w, to);
            at++;
            uint32_t addr[16];
            reg_lds_addr<T, LOGT>(from, addr);
            if (xposed) __syncthreads();   // every wave has read the previous layout
#pragma unroll
            for (int i = 0; i < 16; i++) L::st(addr[i], v[i]);
            __syncthreads();
            reg_lds_addr<T, LOGT>(to, addr);
#pragma unroll
            for (int i = 0; i < 16; i++) v[i] = L::ld(addr[i]);
            xposed = true;
        }
    }
    // store in the final layout
    {
        uint64_t toff = 0;
#pragma unroll
        for (int bt = 0; bt < LOGT; bt++)
            if ((tid >> bt) & 1) toff |= uint64_t(1) << ra.tq[ra.store_pos[bt]];
        uint64_t ib[4];
#pragma unroll
        for (int x = 0; x < 4; x++) ib[x] = uint64_t(1) << ra.tq[ra.store_pos[LOGT + x]];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            uint64_t a = base | toff;
#pragma unroll
            for (int x = 0; x < 4; x++)
                if ((i >> x) & 1) a |= ib[x];
            if (nt) st_stream(st + a, v[i]);
            else st[a] = v[i];
        }
    }
}

// --------------------------------------------------------- strided sweep
template <typename T, int K>
__global__ void __launch_bounds__(NT) k_sweep(Cx<T> *__restrict__ state, uint64_t sstride, int n,
                                              DevOp op, const Cx<T> *__restrict__ cf,
                                              uint64_t cstride, const int32_t *__restrict__ status) {
    constexpr int D = 1 << K;
    if (status && status[blockIdx.y] != 0) return;
    Cx<T> *st = state + size_t(blockIdx.y) * sstride;
    cf += size_t(blockIdx.y) * cstride;
    int p[K];
#pragma unroll
    for (int j = 0; j < K; j++) p[j] = op.pos[j];
    uint64_t off[D];
    off[0] = 0;
#pragma unroll
    for (int r = 1; r < D; r++) off[r] = off[r & (r - 1)] + (uint64_t(1) << p[__builtin_ctz(r)]);
    const uint64_t ngroups = uint64_t(1) << (n - K);
    for (uint64_t g = uint64_t(blockIdx.x) * NT + threadIdx.x; g < ngroups;
         g += uint64_t(gridDim.x) * NT) {
        uint64_t base = g;
#pragma unroll
        for (int j = 0; j < K; j++)
            base = ((base >> p[j]) << (p[j] + 1)) | (base & ((uint64_t(1) << p[j]) - 1));
        Cx<T> x[D], y[D];
#pragma unroll
        for (int r = 0; r < D; r++) x[r] = st[base + off[r]];
        apply_group<T, K>(x, y, op.present, cf + op.coef);
#pragma unroll
        for (int r = 0; r < D; r++) st[base + off[r]] = y[r];
    }
}

// ------------------------------------------------- dense MFMA contraction
// A dense fused operator on KQ = 4 or 5 qubits of a complex64 state, as a
// real-embedded contraction on the FP32 matrix cores: with M = Mr + i Mi,
//     [Yr; Yi] = [[Mr, -Mi], [Mi, Mr]] [Xr; Xi]
// a 2D x 2D real matrix (D = 2^KQ) applied to 32 groups at once by
// v_mfma_f32_32x32x2f32 (32 x 32 outputs += 32 x 2 times 2 x 32), D steps
// of two real rows of the group vectors.  Lane l serves group l mod 32 of
// the wave's 32 and holds its amplitudes 2j + l/32, j < D/2 (the B operand
// of step s is row 2s + l/32 of [Xr; Xi]); it also holds, for each 32-row
// block of the real matrix, entry (32 b + l mod 32, 2s + l/32) of step s
// (the A operand), built once from the operator's XOR-shift diagonals.  The
// accumulator of 32-row block b holds output row 32 b + 8 (r / 4) +
// 4 (l / 32) + r mod 4 of group l mod 32 in register r, so every lane ends
// with the real and imaginary parts of whole output amplitudes.
typedef float F16v __attribute__((ext_vector_type(16)));

template <int KQ>
__global__ void __launch_bounds__(NT) k_dense_mfma(Cx<float> *__restrict__ state, uint64_t sstride, int n,
                                                   DevOp op, const Cx<float> *__restrict__ cf, uint64_t cstride,
                                                   const int32_t *__restrict__ status) {
    constexpr int D = 1 << KQ;
    constexpr int NRB = (2 * D) / 32;
    constexpr int H = D / 2;
    if (status && status[blockIdx.y] != 0) return;
    Cx<float> *st = state + size_t(blockIdx.y) * sstride;
    const Cx<float> *c = cf + size_t(blockIdx.y) * cstride + op.coef;
    const int lane = threadIdx.x & 63, nn = lane & 31, kk = lane >> 5;
    int p[KQ];
#pragma unroll
    for (int j = 0; j < KQ; j++) p[j] = op.pos[j];
    // the operator's coefficients, staged in LDS once per workgroup: the A
    // operands below read each of them on many lanes
    __shared__ Cx<float> cs[D * D];
    const int nterm = __builtin_popcount(op.present);
    for (int x = int(threadIdx.x); x < nterm * D; x += NT) cs[x] = c[x];
    __syncthreads();
    // A operand of every step and row block: real embedding of M[r][col],
    // M[r][col] = d_m[r] for the XOR shift m = r ^ col when present
    float a[NRB][D];
#pragma unroll
    for (int rb = 0; rb < NRB; rb++) {
#pragma unroll
        for (int s = 0; s < D; s++) {
            const int R = rb * 32 + nn, Cc = 2 * s + kk;
            const int r = R % D, col = Cc % D;
            const int m = r ^ col;
            float re = 0.f, im = 0.f;
            if ((op.present >> m) & 1u) {
                const int t = __builtin_popcount(op.present & ((1u << m) - 1u));
                const Cx<float> v = cs[t * D + r];
                re = v.re;
                im = v.im;
            }
            a[rb][s] = (R < D) ? (Cc < D ? re : -im) : (Cc < D ? im : re);
        }
    }
    auto offset = [&](int r) {
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < KQ; j++)
            if ((r >> j) & 1) o |= uint64_t(1) << p[j];
        return o;
    };
    const uint64_t nblk = (uint64_t(1) << (n - KQ)) / 32;
    const uint64_t nwaves = uint64_t(gridDim.x) * (NT / 64);
    for (uint64_t bg = uint64_t(blockIdx.x) * (NT / 64) + (threadIdx.x >> 6); bg < nblk; bg += nwaves) {
        uint64_t base = bg * 32 + uint64_t(nn);
#pragma unroll
        for (int j = 0; j < KQ; j++)
            base = ((base >> p[j]) << (p[j] + 1)) | (base & ((uint64_t(1) << p[j]) - 1));
        Cx<float> x[H];
#pragma unroll
        for (int j = 0; j < H; j++) x[j] = st[base + offset(2 * j + kk)];
        F16v acc[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; rb++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[rb][r] = 0.f;
#pragma unroll
        for (int s = 0; s < D; s++) {
            const float bv = s < H ? x[s].re : x[s - H].im;
#pragma unroll
            for (int rb = 0; rb < NRB; rb++)
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rb][s], bv, acc[rb], 0, 0, 0);
        }
        if constexpr (D == 32) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int i = 8 * (r >> 2) + 4 * kk + (r & 3);
                st[base + offset(i)] = Cx<float>{acc[0][r], acc[1][r]};
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                st[base + offset(4 * kk + r)] = Cx<float>{acc[0][r], acc[0][r + 8]};
                st[base + offset(8 + 4 * kk + r)] = Cx<float>{acc[0][r + 4], acc[0][r + 12]};
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_init_zero(Cx<T> *__restrict__ state, uint64_t sstride,
                                                  uint64_t len) {
    Cx<T> *st = state + size_t(blockIdx.y) * sstride;
    for (uint64_t i = uint64_t(blockIdx.x) * NT + threadIdx.x; i < len; i += uint64_t(gridDim.x) * NT)
        st[i] = Cx<T>{T(i == 0 ? 1 : 0), T(0)};
}

template <typename T>
__global__ void __launch_bounds__(NT) k_collapse(Cx<T> *__restrict__ state, uint64_t len, int q,
                                                 int outcome, T scale) {
    for (uint64_t i = uint64_t(blockIdx.x) * NT + threadIdx.x; i < len; i += uint64_t(gridDim.x) * NT) {
        Cx<T> a = state[i];
        if (int((i >> q) & 1) == outcome) { a.re *= scale; a.im *= scale; }
        else a = Cx<T>{T(0), T(0)};
        state[i] = a;
    }
}

// ------------------------------------------------------- streaming copy
// The same-footprint ceiling of a tile pass: workgroup b moves 64 KiB block
// (b + rotate) mod nblocks of src to dst, 256 threads, 16 elements of 16
// bytes each, all loads in flight before the first store (the tile kernel's
// grid shape and access order for complex128).  dst may equal src: an
// in-place pass then reads and writes every byte once, the traffic of one
// tile pass.  Changing `rotate` between calls hands each block to another
// workgroup, and so to another XCD's L2, as a tile pass over new qubits does.
template <bool NTMP>
__global__ void __launch_bounds__(256) k_stream_copy(const uint32_t *src, uint32_t *dst, uint64_t n16,
                                                     uint32_t nblocks, uint32_t rotate) {
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    const U4 *s = reinterpret_cast<const U4 *>(src);
    U4 *d = reinterpret_cast<U4 *>(dst);
    const uint64_t blk = (uint64_t(blockIdx.x) + rotate) % nblocks;
    const uint64_t base = blk * 4096 + threadIdx.x;
    U4 v[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const uint64_t x = base + uint64_t(i) * 256;
        if (x < n16) v[i] = NTMP ? __builtin_nontemporal_load(s + x) : s[x];
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const uint64_t x = base + uint64_t(i) * 256;
        if (x < n16) {
            if (NTMP) __builtin_nontemporal_store(v[i], d + x);
            else d[x] = v[i];
        }
    }
}

// ---------------------------------------------------------- reductions
struct MargArgs {
    int32_t n, nqs;
    int32_t sorted[12];   // qubits of the marginal, ascending (for zero insertion)
    int32_t qs[12];       // qubits in output-bit order
};

// partials[((b * nbins) + bin) * nchunks + chunk]
template <typename T>
__global__ void __launch_bounds__(NT) k_marginal(const Cx<T> *__restrict__ state, uint64_t sstride,
                                                 MargArgs a, double *__restrict__ partials) {
    const Cx<T> *st = state + size_t(blockIdx.z) * sstride;
    const uint32_t bin = blockIdx.y, chunk = blockIdx.x, nchunks = gridDim.x;
    const uint64_t R = uint64_t(1) << (a.n - a.nqs);
    const uint64_t per = R / nchunks;
    uint64_t binbits = 0;
    for (int i = 0; i < a.nqs; i++)
        if ((bin >> i) & 1) binbits |= uint64_t(1) << a.qs[i];
    double acc[1] = {0.0};
    for (uint64_t r = uint64_t(chunk) * per + threadIdx.x; r < uint64_t(chunk + 1) * per; r += NT) {
        uint64_t x = r;
        for (int i = 0; i < a.nqs; i++) {
            const int p = a.sorted[i];
            x = ((x >> p) << (p + 1)) | (x & ((uint64_t(1) << p) - 1));
        }
        acc[0] += norm2(st[x | binbits]);
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0)
        partials[(size_t(blockIdx.z) * gridDim.y + bin) * nchunks + chunk] = acc[0];
}

// Pauli overlaps of up to kPauliRow terms that share an X mask (one row of
// the table built by pauli_rows), S_k = sum_x s_k(x) conj(a[x ^ X]) a[x] with
// s_k(x) = (-1)^popcount(x & z_k).  For X != 0 the sum runs over the pairs
// {x, x ^ X} with bit h of x clear (h the highest bit of X), each amplitude
// read once: with p = conj(a[x ^ X]) a[x], the pair adds
// s_k(x) (p + sigma_k conj(p)), sigma_k = (-1)^popcount(X & z_k), which is
// 2 s_k(x) Re p when sigma_k = 1 and 2i s_k(x) Im p otherwise.  For X = 0,
// S_k = sum_x s_k(x) |a[x]|^2.  Each term's sums run in the same order as
// they would alone.
// partials[((b * nterms + k) * 2 + comp) * nchunks + chunk]
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_pauli(const Cx<T> *__restrict__ state, uint64_t sstride,
                                              int n, const uint64_t *__restrict__ zmask,
                                              const uint64_t *__restrict__ rows, uint32_t nterms,
                                              double *__restrict__ partials) {
    const Cx<T> *st = state + size_t(blockIdx.z) * sstride;
    const uint32_t chunk = blockIdx.x, nchunks = gridDim.x;
    const uint64_t *row = rows + size_t(blockIdx.y) * (2 + kPauliRow);
    const uint64_t xm = row[0];
    const int cnt = int(row[1]);
    uint64_t z[R];
#pragma unroll
    for (int j = 0; j < R; j++) z[j] = j < cnt ? zmask[row[2 + j]] : 0;
    double acc[2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; j++) acc[j] = 0.0;
    if (xm == 0) {
        const uint64_t per = (uint64_t(1) << n) / nchunks;
        for (uint64_t x = uint64_t(chunk) * per + threadIdx.x; x < uint64_t(chunk + 1) * per; x += NT) {
            const double w = norm2(st[x]);
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (j < cnt) {
                    const bool odd = __builtin_popcountll(x & z[j]) & 1;
                    acc[2 * j] += odd ? -w : w;
                }
            }
        }
    } else {
        const int h = 63 - __builtin_clzll(xm);
        const uint64_t lowm = (uint64_t(1) << h) - 1;
        bool real_part[R];
#pragma unroll
        for (int j = 0; j < R; j++) real_part[j] = !(__builtin_popcountll(xm & z[j]) & 1);
        const uint64_t per = (uint64_t(1) << (n - 1)) / nchunks;
        for (uint64_t y = uint64_t(chunk) * per + threadIdx.x; y < uint64_t(chunk + 1) * per; y += NT) {
            const uint64_t x = ((y >> h) << (h + 1)) | (y & lowm);
            const Cx<T> a = st[x], c = st[x ^ xm];
            const double ar = double(a.re), ai = double(a.im), cr = double(c.re), ci = double(c.im);
            // 2 conj(c) * a
            const double re = 2.0 * (cr * ar + ci * ai), im = 2.0 * (cr * ai - ci * ar);
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (j < cnt) {
                    const bool odd = __builtin_popcountll(x & z[j]) & 1;
                    if (real_part[j]) acc[2 * j] += odd ? -re : re;
                    else acc[2 * j + 1] += odd ? -im : im;
                }
            }
        }
    }
    block_sum<2 * R>(acc);
    if (threadIdx.x == 0) {
        for (int j = 0; j < cnt; j++) {
            const size_t o = (size_t(blockIdx.z) * nterms + size_t(row[2 + j])) * 2;
            partials[(o + 0) * nchunks + chunk] = acc[2 * j];
            partials[(o + 1) * nchunks + chunk] = acc[2 * j + 1];
        }
    }
}

// out[i] = sum_{c < nchunks} partials[i * nchunks + c], in index order.
__global__ void __launch_bounds__(NT) k_finish(const double *__restrict__ partials, uint32_t nchunks,
                                               double *__restrict__ out) {
    const double *p = partials + size_t(blockIdx.x) * nchunks;
    double acc[1] = {0.0};
    for (uint32_t c = threadIdx.x; c < nchunks; c += NT) acc[0] += p[c];
    block_sum<1>(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc[0];
}

// ------------------------------------------------- batched measurement
// Measurement, assertion, reset, or measurement then reset, of qubit q in
// every state of a batch whose state does not fit one tile: P0, P1 come from
// a marginal reduction (p01[2b], p01[2b+1]); every thread takes the same
// decision from them and updates its amplitude pairs (x, x | 2^q).
template <typename T>
__global__ void __launch_bounds__(NT) k_decide(Cx<T> *__restrict__ state, uint64_t sstride, int n,
                                               int q, int kind, int slot,
                                               const double *__restrict__ p01, MeasArgs ma) {
    const uint32_t b = blockIdx.y;
    if (ma.status && ma.status[b] != 0) return;
    const double P0 = p01[2 * b], P1 = p01[2 * b + 1];
    int o = 0, fail = 0;
    bool swap = false, touch = true;
    const bool to_zero = kind == qs::DEVOP_MEASURE_RESET;   // the outcome then moves to |0>
    double kept = 1.0;
    const size_t idx = size_t(b) * ma.nslots + slot;
    if (kind == qs::DEVOP_RESET) {
        if (P1 == 0.0) touch = false;
        else if (P0 == 0.0) swap = true;
        else fail = QSIM_E_NOT_DEFINITE;
    } else {
        if (kind == qs::DEVOP_ASSERT0) {
            if (!(P0 > 0.0)) fail = QSIM_E_ZERO_PROB;
        } else if (ma.forced && ma.forced[idx] >= 0) {
            o = ma.forced[idx];
            if (!((o ? P1 : P0) > 0.0)) fail = QSIM_E_ZERO_PROB;
        } else {
            o = (ma.uniforms[idx] < P0 / (P0 + P1)) ? 0 : 1;
        }
        kept = o ? P1 : P0;
    }
    if (fail) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ma.status[b] = fail;
            if (ma.fail_at) ma.fail_at[b] = -2 - slot;
        }
        return;
    }
    if (kind != qs::DEVOP_RESET && blockIdx.x == 0 && threadIdx.x == 0) {
        ma.outcomes[idx] = o;
        ma.probs[idx] = kept / (P0 + P1);
    }
    if (!touch) return;
    const T scale = T(1.0 / sqrt(kept));
    Cx<T> *st = state + size_t(b) * sstride;
    const uint64_t half = uint64_t(1) << (n - 1), bq = uint64_t(1) << q;
    for (uint64_t g = uint64_t(blockIdx.x) * NT + threadIdx.x; g < half; g += uint64_t(gridDim.x) * NT) {
        const uint64_t x0 = ((g >> q) << (q + 1)) | (g & (bq - 1)), x1 = x0 | bq;
        const Cx<T> a0 = st[x0], a1 = st[x1];
        Cx<T> n0, n1 = Cx<T>{T(0), T(0)};
        if (swap) n0 = a1;
        else if (o == 0) n0 = Cx<T>{a0.re * scale, a0.im * scale};
        else if (to_zero) n0 = Cx<T>{a1.re * scale, a1.im * scale};
        else { n0 = Cx<T>{T(0), T(0)}; n1 = Cx<T>{a1.re * scale, a1.im * scale}; }
        st[x0] = n0;
        st[x1] = n1;
    }
}

// Per-state operator coefficients of a parameterised template: entry e
// covers `count` coefficients; with np angle slots its template holds 2^np
// blocks, block s weighted by prod_j (bit j of s ? sin : cos)(theta_slot_j / 2).
template <typename T>
__global__ void __launch_bounds__(NT) k_bind(const double *__restrict__ tmpl,
                                             const BindEntry *__restrict__ ents,
                                             const double *__restrict__ params, int nparams,
                                             Cx<T> *__restrict__ out, uint64_t cstride,
                                             uint32_t nstates) {
    const BindEntry e = ents[blockIdx.x];
    const uint64_t total = uint64_t(nstates) * e.count;
    for (uint64_t idx = uint64_t(blockIdx.y) * NT + threadIdx.x; idx < total;
         idx += uint64_t(gridDim.y) * NT) {
        const uint32_t b = uint32_t(idx / e.count), c = uint32_t(idx % e.count);
        double cs[3], sn[3];
        for (int j = 0; j < e.np; j++) {
            const double th = params[size_t(b) * nparams + e.slot[j]];
            cs[j] = cos(0.5 * th);
            sn[j] = sin(0.5 * th);
        }
        double re = 0.0, im = 0.0;
        for (int sb = 0; sb < (1 << e.np); sb++) {
            double w = 1.0;
            for (int j = 0; j < e.np; j++) w *= ((sb >> j) & 1) ? sn[j] : cs[j];
            const size_t src = 2 * (size_t(e.tmpl_off) + size_t(sb) * e.count + c);
            re += w * tmpl[src];
            im += w * tmpl[src + 1];
        }
        out[size_t(b) * cstride + e.bound_off + c] = Cx<T>{T(re), T(im)};
    }
}

__global__ void __launch_bounds__(NT) k_fill_i32(int32_t *__restrict__ p, int32_t v, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += uint64_t(gridDim.x) * NT) p[i] = v;
}

// -------------------------------------------------------------- sampling
// Inclusive prefix sums of |a_x|^2 in FP64, in three fixed-order steps:
// per-block local scans (4096 elements per block, 16 per thread), block
// totals scanned on the host, block offsets added back.
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_BLOCK = NT * SCAN_PER_THREAD;

template <typename T>
__global__ void __launch_bounds__(NT) k_blockscan(const Cx<T> *__restrict__ state, uint64_t len,
                                                  double *__restrict__ cum, double *__restrict__ bsum) {
    __shared__ double tsum[NT];
    const uint64_t b0 = uint64_t(blockIdx.x) * SCAN_BLOCK + uint64_t(threadIdx.x) * SCAN_PER_THREAD;
    double loc[SCAN_PER_THREAD];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; i++) {
        const uint64_t x = b0 + i;
        run += (x < len) ? norm2(state[x]) : 0.0;
        loc[i] = run;
    }
    tsum[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int j = 0; j < NT; j++) {
            const double v = tsum[j];
            tsum[j] = acc;    // exclusive prefix of thread totals
            acc += v;
        }
        bsum[blockIdx.x] = acc;
    }
    __syncthreads();
    const double off = tsum[threadIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; i++) {
        const uint64_t x = b0 + i;
        if (x < len) cum[x] = off + loc[i];
    }
}

__global__ void __launch_bounds__(NT) k_addoff(double *__restrict__ cum, uint64_t len,
                                               const double *__restrict__ boff) {
    for (uint64_t x = uint64_t(blockIdx.x) * NT + threadIdx.x; x < len; x += uint64_t(gridDim.x) * NT)
        cum[x] += boff[x / SCAN_BLOCK];
}

// Shot s: smallest x with cum[x] > u[s] * cum[len - 1].
__global__ void __launch_bounds__(NT) k_search(const double *__restrict__ cum, uint64_t len,
                                               const double *__restrict__ u, uint64_t m,
                                               uint64_t *__restrict__ out) {
    const uint64_t s = uint64_t(blockIdx.x) * NT + threadIdx.x;
    if (s >= m) return;
    const double target = u[s] * cum[len - 1];
    uint64_t lo = 0, hi = len - 1;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    out[s] = lo;
}

// ------------------------------------------------------------- launchers
namespace {
int check(hipError_t e) { return note_hip(e, "kernel launch"); }

uint32_t grid_for(uint64_t work) {
    uint64_t g = (work + NT - 1) / NT;
    if (g > 65536) g = 65536;
    return uint32_t(g ? g : 1);
}
}  // namespace

size_t max_lds_bytes() { return 160 * 1024; }

// The tile kernel addresses its LDS from byte 0: it must have no static LDS.
static int tile_static_lds = 0;

template <typename T, int LE, int TNT>
static void lds_attr() {
    const void *f = reinterpret_cast<const void *>(&k_tile<T, LE, TNT>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(max_lds_bytes()));
    if (e != hipSuccess) note_hip(e, "hipFuncSetAttribute(k_tile)");
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, f) == hipSuccess && fa.sharedSizeBytes != 0) tile_static_lds = 1;
}

template <typename T, int LOGT>
static void reg_attr() {
    const void *f = reinterpret_cast<const void *>(&k_reg<T, LOGT>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(max_lds_bytes()));
    if (e != hipSuccess) note_hip(e, "hipFuncSetAttribute(k_reg)");
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, f) == hipSuccess && fa.sharedSizeBytes != 0) tile_static_lds = 1;
}

int init_kernels() {
    static int done = 0;
    if (done) return QSIM_OK;
    reg_attr<float, 6>();
    reg_attr<float, 7>();
    reg_attr<float, 8>();
    reg_attr<float, 9>();
    reg_attr<double, 6>();
    reg_attr<double, 7>();
    reg_attr<double, 8>();
    reg_attr<double, 9>();
    // Allow the tile kernels the largest dynamic LDS they use (160 KiB).  The
    // attribute is advisory on this platform: a refusal is recorded, and a
    // launch that then asks for too much LDS reports its own error.
    lds_attr<float, 0, 256>();
    lds_attr<float, 1, 256>();
    lds_attr<float, 2, 256>();
    lds_attr<float, 3, 256>();
    lds_attr<float, 4, 256>();
    lds_attr<float, 5, 256>();
    lds_attr<float, 6, 256>();
    lds_attr<float, 0, 512>();
    lds_attr<float, 1, 512>();
    lds_attr<float, 2, 512>();
    lds_attr<float, 3, 512>();
    lds_attr<float, 4, 512>();
    lds_attr<float, 5, 512>();
    lds_attr<float, 6, 512>();
    lds_attr<double, 0, 256>();
    lds_attr<double, 1, 256>();
    lds_attr<double, 2, 256>();
    lds_attr<double, 3, 256>();
    lds_attr<double, 4, 256>();
    lds_attr<double, 5, 256>();
    lds_attr<double, 6, 256>();
    lds_attr<double, 0, 512>();
    lds_attr<double, 1, 512>();
    lds_attr<double, 2, 512>();
    lds_attr<double, 3, 512>();
    lds_attr<double, 4, 512>();
    lds_attr<double, 5, 512>();
    lds_attr<double, 6, 512>();
    (void)hipGetLastError();
    if (tile_static_lds) {
        note_hip(hipErrorInvalidKernelFile, "k_tile declares static LDS (its tile must start at LDS byte 0)");
        return QSIM_E_UNSUPPORTED;
    }
    done = 1;
    return QSIM_OK;
}

template <typename T, int LE, int TNT>
static void tile_t(void *state, uint64_t sstride, uint32_t nstates, const TileArgs &ta,
                   const DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb,
                   uint32_t ce, uint64_t cstride, const MeasArgs &m, uint32_t flags,
                   hipStream_t st) {
    const dim3 grid(uint32_t(uint64_t(1) << (ta.n - ta.t)), nstates);
    const size_t lds = tile_lds_bytes(sizeof(Cx<T>), ta.t, oe - ob, ce - cb);
    hipLaunchKernelGGL((k_tile<T, LE, TNT>), grid, dim3(TNT), lds, st, (Cx<T> *)state, sstride, ta,
                       ops, ob, oe, (const Cx<T> *)coefs, cb, ce, cstride, m, flags);
}

template <typename T, int TNT>
static int tile_dispatch_t(void *state, uint64_t sstride, uint32_t nstates, const TileArgs &ta,
                           const DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs,
                           uint32_t cb, uint32_t ce, uint64_t cstride, const MeasArgs &m,
                           uint32_t flags, hipStream_t st) {
    constexpr int LOGT = (TNT == 512) ? 9 : 8;
    const int le = ta.t > LOGT ? ta.t - LOGT : 0;
#define QK_TILE_CASE(L)                                                                              \
    case L: tile_t<T, L, TNT>(state, sstride, nstates, ta, ops, ob, oe, coefs, cb, ce, cstride, m, flags, st); break;
    switch (le) {
        QK_TILE_CASE(0)
        QK_TILE_CASE(1)
        QK_TILE_CASE(2)
        QK_TILE_CASE(3)
        QK_TILE_CASE(4)
        QK_TILE_CASE(5)
        QK_TILE_CASE(6)
    default: return QSIM_E_ARG;
    }
#undef QK_TILE_CASE
    return QSIM_OK;
}

template <typename T>
static int tile_dispatch(void *state, uint64_t sstride, uint32_t nstates, const TileArgs &ta,
                         const DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs,
                         uint32_t cb, uint32_t ce, uint64_t cstride, const MeasArgs &m,
                         uint32_t flags, hipStream_t st) {
    if (ta.threads == 512)
        return tile_dispatch_t<T, 512>(state, sstride, nstates, ta, ops, ob, oe, coefs, cb, ce, cstride, m, flags, st);
    return tile_dispatch_t<T, 256>(state, sstride, nstates, ta, ops, ob, oe, coefs, cb, ce, cstride, m, flags, st);
}

size_t tile_lds_bytes(size_t elem, int t, uint32_t nrec, uint32_t ncoef) {
    return (size_t(1) << t) * elem + kTileRedBytes + size_t(nrec) * sizeof(DevOp) + size_t(ncoef) * elem;
}

int launch_tile(int dtype, void *state, uint64_t sstride, uint32_t nstates, const TileArgs &ta,
                const DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb,
                uint32_t ce, uint64_t cstride, const MeasArgs *ma, uint32_t flags,
                hipStream_t st) {
    MeasArgs m{};
    if (ma) m = *ma;
    if (ta.t < 1 || ta.t > 14 || ta.t > ta.n || ce < cb || oe < ob || (ta.threads != 256 && ta.threads != 512))
        return QSIM_E_ARG;
    if (tile_lds_bytes(dtype == QSIM_C64 ? 8 : 16, ta.t, oe - ob, ce - cb) > max_lds_bytes())
        return QSIM_E_CAPACITY;
    int rc = (dtype == QSIM_C64)
                 ? tile_dispatch<float>(state, sstride, nstates, ta, ops, ob, oe, coefs, cb, ce, cstride, m, flags, st)
                 : tile_dispatch<double>(state, sstride, nstates, ta, ops, ob, oe, coefs, cb, ce, cstride, m, flags, st);
    if (rc) return rc;
    return check(hipGetLastError());
}

template <typename T, int LOGT>
static void reg_t(void *state, uint64_t sstride, uint32_t nstates, const RegArgs &ra, const DevOp *ops,
                  uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb, uint32_t ce, uint64_t cstride,
                  const int32_t *status, uint32_t flags, size_t lds, hipStream_t st) {
    const dim3 grid(uint32_t(uint64_t(1) << (ra.n - ra.t)), nstates);
    hipLaunchKernelGGL((k_reg<T, LOGT>), grid, dim3(1 << LOGT), lds, st, (Cx<T> *)state, sstride, ra, ops, ob,
                       oe, (const Cx<T> *)coefs, cb, ce, cstride, status, flags);
}

size_t reg_lds_bytes(size_t elem, int t, bool relayouts, uint32_t nrec) {
    return (relayouts ? (elem << t) : size_t(0)) + size_t(nrec) * sizeof(DevOp);
}

int launch_reg(int dtype, void *state, uint64_t sstride, uint32_t nstates, const RegArgs &ra,
               const DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb, uint32_t ce,
               uint64_t cstride, const int32_t *status, uint32_t flags, hipStream_t st) {
    const int logt = ra.t - 4;
    const size_t elem = dtype == QSIM_C64 ? 8 : 16;
    if (logt < 6 || logt > 9 || ra.t >= ra.n || ra.n - ra.t > 31 || oe < ob || ce < cb ||
        (ra.lds_bytes != reg_lds_bytes(elem, ra.t, false, oe - ob) &&
                                          ra.lds_bytes != reg_lds_bytes(elem, ra.t, true, oe - ob)))
        return QSIM_E_ARG;
    if (ra.lds_bytes > max_lds_bytes()) return QSIM_E_CAPACITY;
    const size_t lds = ra.lds_bytes;
    if (dtype == QSIM_C64) {
        switch (logt) {
        case 6: reg_t<float, 6>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        case 7: reg_t<float, 7>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        case 8: reg_t<float, 8>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        default: reg_t<float, 9>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        }
    } else {
        switch (logt) {
        case 6: reg_t<double, 6>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        case 7: reg_t<double, 7>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        case 8: reg_t<double, 8>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        default: reg_t<double, 9>(state, sstride, nstates, ra, ops, ob, oe, coefs, cb, ce, cstride, status, flags, lds, st); break;
        }
    }
    return check(hipGetLastError());
}

template <typename T>
static void sweep_t(Cx<T> *state, uint64_t sstride, uint32_t nstates, int n, const DevOp &op,
                    const Cx<T> *cf, uint64_t cstride, const int32_t *status, hipStream_t st) {
    const dim3 grid(grid_for(uint64_t(1) << (n - op.k)), nstates);
    switch (op.k) {
    case 1: hipLaunchKernelGGL((k_sweep<T, 1>), grid, dim3(NT), 0, st, state, sstride, n, op, cf, cstride, status); break;
    case 2: hipLaunchKernelGGL((k_sweep<T, 2>), grid, dim3(NT), 0, st, state, sstride, n, op, cf, cstride, status); break;
    case 3: hipLaunchKernelGGL((k_sweep<T, 3>), grid, dim3(NT), 0, st, state, sstride, n, op, cf, cstride, status); break;
    case 4: hipLaunchKernelGGL((k_sweep<T, 4>), grid, dim3(NT), 0, st, state, sstride, n, op, cf, cstride, status); break;
    default: hipLaunchKernelGGL((k_sweep<T, 5>), grid, dim3(NT), 0, st, state, sstride, n, op, cf, cstride, status); break;
    }
}

bool dense_mfma_ok(int dtype, int n, const DevOp &op) {
    static const int enabled = [] {
        const char *v = std::getenv("QSIM_MFMA");
        return v ? std::atoi(v) : 1;
    }();
    if (!enabled || dtype != QSIM_C64 || (op.k != 4 && op.k != 5) || n - op.k < 5) return false;
    // the contraction does the dense work: worth it when at least half of the
    // XOR diagonals are present
    return __builtin_popcount(op.present) * 2 >= (1 << op.k);
}

int launch_sweep(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n,
                 const DevOp &op, const void *coefs, hipStream_t st, uint64_t cstride,
                 const int32_t *status) {
    if (op.k < 1 || op.k > 5 || op.k > n) return QSIM_E_ARG;
    if (dense_mfma_ok(dtype, n, op)) {
        const uint64_t nblk = (uint64_t(1) << (n - op.k)) / 32;   // 32 groups per wave
        const uint64_t blocks = std::min<uint64_t>((nblk + 3) / 4, 8192);
        const dim3 grid(uint32_t(blocks), nstates);
        if (op.k == 5)
            hipLaunchKernelGGL(k_dense_mfma<5>, grid, dim3(NT), 0, st, (Cx<float> *)state, sstride, n, op,
                               (const Cx<float> *)coefs, cstride, status);
        else
            hipLaunchKernelGGL(k_dense_mfma<4>, grid, dim3(NT), 0, st, (Cx<float> *)state, sstride, n, op,
                               (const Cx<float> *)coefs, cstride, status);
        return check(hipGetLastError());
    }
    if (dtype == QSIM_C64)
        sweep_t<float>((Cx<float> *)state, sstride, nstates, n, op, (const Cx<float> *)coefs, cstride, status, st);
    else
        sweep_t<double>((Cx<double> *)state, sstride, nstates, n, op, (const Cx<double> *)coefs, cstride, status, st);
    return check(hipGetLastError());
}

int launch_init_zero(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n,
                     hipStream_t st) {
    const uint64_t len = uint64_t(1) << n;
    const dim3 grid(grid_for(len), nstates);
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_init_zero<float>, grid, dim3(NT), 0, st, (Cx<float> *)state, sstride, len);
    else
        hipLaunchKernelGGL(k_init_zero<double>, grid, dim3(NT), 0, st, (Cx<double> *)state, sstride, len);
    return check(hipGetLastError());
}

int launch_stream_copy(void *dst, const void *src, uint64_t bytes, bool nontemporal, uint32_t rotate,
                       hipStream_t st) {
    const uint64_t n16 = bytes / 16;
    if (n16 == 0) return QSIM_OK;
    const uint64_t nb = (n16 + 4095) / 4096;
    if (nb > 0x7fffffffull) return QSIM_E_ARG;
    const uint32_t nblocks = uint32_t(nb);
    if (nontemporal)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3(nblocks), dim3(256), 0, st, (const uint32_t *)src,
                           (uint32_t *)dst, n16, nblocks, rotate % nblocks);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3(nblocks), dim3(256), 0, st, (const uint32_t *)src,
                           (uint32_t *)dst, n16, nblocks, rotate % nblocks);
    return check(hipGetLastError());
}

uint32_t marginal_chunks(int n, int nqs) {
    const uint64_t R = uint64_t(1) << (n - nqs);
    uint64_t c = R / 4096;
    if (c < 1) c = 1;
    if (c > 512) c = 512;
    return uint32_t(c);
}

int launch_marginal(int dtype, const void *state, uint64_t sstride, uint32_t nstates, int n,
                    const int *qs, int nqs, double *partials, double *out, hipStream_t st,
                    uint32_t nchunks_override) {
    if (nqs < 0 || nqs > 12 || nqs > n) return QSIM_E_ARG;
    MargArgs a{};
    a.n = n;
    a.nqs = nqs;
    for (int i = 0; i < nqs; i++) a.qs[i] = a.sorted[i] = qs[i];
    for (int i = 0; i < nqs; i++)
        for (int j = i + 1; j < nqs; j++)
            if (a.sorted[j] < a.sorted[i]) { int t = a.sorted[i]; a.sorted[i] = a.sorted[j]; a.sorted[j] = t; }
    uint32_t nchunks = marginal_chunks(n, nqs);
    if (nchunks_override && nchunks_override < nchunks) nchunks = nchunks_override;
    const dim3 grid(nchunks, 1u << nqs, nstates);
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_marginal<float>, grid, dim3(NT), 0, st, (const Cx<float> *)state, sstride, a, partials);
    else
        hipLaunchKernelGGL(k_marginal<double>, grid, dim3(NT), 0, st, (const Cx<double> *)state, sstride, a, partials);
    hipLaunchKernelGGL(k_finish, dim3(uint32_t(nstates) << nqs), dim3(NT), 0, st, partials, nchunks, out);
    return check(hipGetLastError());
}

// ------------------------------------------- allocation-free marginals
// Reduction scratch of launch_probs_noalloc: a fixed device array, one copy
// per GPU, that lives until the process ends.  Host code never uses its name
// as an address: the device address comes from hipGetSymbolAddress, once per
// device, and only that pointer reaches the kernels.
constexpr uint32_t kScratchPartials = 1u << 17;            // doubles of chunk partials
constexpr uint32_t kScratchDoubles = kScratchPartials + 4096;
static __device__ __align__(256) double scratch[kScratchDoubles];

// out[j] = raw[j] / sum_j raw[j], the sum taken in index order by one thread
// (the order a host loop over the same values uses).
__global__ void __launch_bounds__(NT) k_normalize(const double *__restrict__ raw, uint32_t m,
                                                  double *__restrict__ out) {
    __shared__ double tot;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (uint32_t j = 0; j < m; j++) s += raw[j];
        tot = s;
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < m; j += NT) out[j] = raw[j] / tot;
}

int launch_probs_noalloc(int dtype, const void *state, int n, const int *qs, int nqs, double *dev_out,
                         hipStream_t st) {
    if (nqs < 0 || nqs > 12 || nqs > n) return QSIM_E_ARG;
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptrs[kMaxDevices] = {};
    int dev = 0;
    int rc = note_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return QSIM_E_ARG;
    double *base;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!ptrs[dev]) {
            void *p = nullptr;
            rc = note_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
            if (rc) return rc;
            ptrs[dev] = static_cast<double *>(p);
        }
        base = ptrs[dev];
    }
    double *partials = base, *raw = base + kScratchPartials;
    const uint32_t cap = kScratchPartials >> nqs;
    const uint32_t nch = marginal_chunks(n, nqs) < cap ? marginal_chunks(n, nqs) : cap;
    rc = launch_marginal(dtype, state, 0, 1, n, qs, nqs, partials, raw, st, nch);
    if (rc) return rc;
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(NT), 0, st, raw, 1u << nqs, dev_out);
    return check(hipGetLastError());
}

uint32_t pauli_chunks(int n) {
    uint64_t c = (uint64_t(1) << n) / 4096;
    if (c < 1) c = 1;
    if (c > 256) c = 256;
    return uint32_t(c);
}

namespace {
int pauli_bucket(size_t cnt) { return cnt > 4 ? 0 : cnt > 2 ? 1 : cnt == 2 ? 2 : 3; }
}  // namespace

PauliRows pauli_rows(const qsim_pauli *t, size_t nt, std::vector<uint64_t> *table) {
    std::vector<uint32_t> idx(nt);
    for (size_t k = 0; k < nt; k++) idx[k] = uint32_t(k);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return t[a].xmask < t[b].xmask; });
    // rows as (first sorted index, count), then ordered by bucket
    std::vector<std::pair<size_t, size_t>> rows;
    for (size_t i = 0; i < nt;) {
        size_t j = i;
        while (j < nt && j - i < size_t(kPauliRow) && t[idx[j]].xmask == t[idx[i]].xmask) j++;
        rows.push_back({i, j - i});
        i = j;
    }
    std::stable_sort(rows.begin(), rows.end(), [](const std::pair<size_t, size_t> &a,
                                                  const std::pair<size_t, size_t> &b) {
        return pauli_bucket(a.second) < pauli_bucket(b.second);
    });
    table->assign(nt, 0);
    for (size_t k = 0; k < nt; k++) (*table)[k] = t[k].zmask;
    PauliRows pr;
    for (const auto &r : rows) {
        table->push_back(t[idx[r.first]].xmask);
        table->push_back(uint64_t(r.second));
        for (int s = 0; s < kPauliRow; s++) table->push_back(size_t(s) < r.second ? idx[r.first + s] : 0);
        pr.bucket[pauli_bucket(r.second)]++;
        pr.rows++;
    }
    return pr;
}

int launch_pauli(int dtype, const void *state, uint64_t sstride, uint32_t nstates, int n,
                 const uint64_t *table, int nterms, const PauliRows &pr, double *partials,
                 double *out, hipStream_t st, uint32_t nchunks_override) {
    if (nterms <= 0) return QSIM_OK;
    const uint32_t nrows = pr.bucket[0] + pr.bucket[1] + pr.bucket[2] + pr.bucket[3];
    if (pr.rows == 0 || nrows != pr.rows || pr.rows > uint32_t(nterms)) return QSIM_E_ARG;
    uint32_t nchunks = pauli_chunks(n);
    if (nchunks_override && nchunks_override < nchunks) nchunks = nchunks_override;
    const uint64_t *rows = table + nterms;
    const int64_t stride = 2 + kPauliRow;
    for (int b = 0; b < 4; b++) {
        if (pr.bucket[b] == 0) {
            continue;
        }
        const dim3 grid(nchunks, pr.bucket[b], nstates);
#define QK_PAULI(R)                                                                                         \
    if (dtype == QSIM_C64)                                                                                  \
        hipLaunchKernelGGL((k_pauli<float, R>), grid, dim3(NT), 0, st, (const Cx<float> *)state, sstride, n, \
                           table, rows, uint32_t(nterms), partials);                                        \
    else                                                                                                    \
        hipLaunchKernelGGL((k_pauli<double, R>), grid, dim3(NT), 0, st, (const Cx<double> *)state, sstride,  \
                           n, table, rows, uint32_t(nterms), partials);
        switch (b) {
        case 0: QK_PAULI(8) break;
        case 1: QK_PAULI(4) break;
        case 2: QK_PAULI(2) break;
        default: QK_PAULI(1) break;
        }
#undef QK_PAULI
        rows += stride * int64_t(pr.bucket[b]);
    }
    hipLaunchKernelGGL(k_finish, dim3(uint32_t(nstates) * uint32_t(nterms) * 2), dim3(NT), 0, st,
                       partials, nchunks, out);
    return check(hipGetLastError());
}

int launch_decide(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n, int q,
                  int kind, int slot, const double *p01, const MeasArgs &ma, hipStream_t st) {
    const dim3 grid(grid_for(uint64_t(1) << (n - 1)) > 1024 ? 1024 : grid_for(uint64_t(1) << (n - 1)), nstates);
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_decide<float>, grid, dim3(NT), 0, st, (Cx<float> *)state, sstride, n, q, kind, slot, p01, ma);
    else
        hipLaunchKernelGGL(k_decide<double>, grid, dim3(NT), 0, st, (Cx<double> *)state, sstride, n, q, kind, slot, p01, ma);
    return check(hipGetLastError());
}

int launch_bind(int dtype, const double *tmpl, const BindEntry *ents, uint32_t nents,
                const double *params, int nparams, void *out, uint64_t cstride, uint32_t nstates,
                uint32_t max_count, hipStream_t st) {
    if (nents == 0) return QSIM_OK;
    uint64_t per = (uint64_t(nstates) * max_count + NT - 1) / NT;
    const dim3 grid(nents, uint32_t(per > 256 ? 256 : (per ? per : 1)));
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_bind<float>, grid, dim3(NT), 0, st, tmpl, ents, params, nparams, (Cx<float> *)out, cstride, nstates);
    else
        hipLaunchKernelGGL(k_bind<double>, grid, dim3(NT), 0, st, tmpl, ents, params, nparams, (Cx<double> *)out, cstride, nstates);
    return check(hipGetLastError());
}

int launch_fill_i32(int32_t *p, int32_t v, uint64_t n, hipStream_t st) {
    if (n == 0) return QSIM_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(NT), 0, st, p, v, n);
    return check(hipGetLastError());
}

uint64_t scan_blocks(int n) { return ((uint64_t(1) << n) + SCAN_BLOCK - 1) / SCAN_BLOCK; }

int launch_blockscan(int dtype, const void *state, int n, double *cum, double *bsum, hipStream_t st) {
    const uint64_t len = uint64_t(1) << n;
    const dim3 grid(uint32_t(scan_blocks(n)));
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_blockscan<float>, grid, dim3(NT), 0, st, (const Cx<float> *)state, len, cum, bsum);
    else
        hipLaunchKernelGGL(k_blockscan<double>, grid, dim3(NT), 0, st, (const Cx<double> *)state, len, cum, bsum);
    return check(hipGetLastError());
}

int launch_addoff_search(double *cum, int n, const double *boff, const double *u, uint64_t m,
                         uint64_t *out, hipStream_t st) {
    const uint64_t len = uint64_t(1) << n;
    hipLaunchKernelGGL(k_addoff, dim3(grid_for(len)), dim3(NT), 0, st, cum, len, boff);
    if (m) hipLaunchKernelGGL(k_search, dim3(uint32_t((m + NT - 1) / NT)), dim3(NT), 0, st, cum, len, u, m, out);
    return check(hipGetLastError());
}

int launch_collapse(int dtype, void *state, int n, int q, int outcome, double scale, hipStream_t st) {
    const uint64_t len = uint64_t(1) << n;
    if (dtype == QSIM_C64)
        hipLaunchKernelGGL(k_collapse<float>, dim3(grid_for(len)), dim3(NT), 0, st, (Cx<float> *)state, len, q, outcome, float(scale));
    else
        hipLaunchKernelGGL(k_collapse<double>, dim3(grid_for(len)), dim3(NT), 0, st, (Cx<double> *)state, len, q, outcome, scale);
    return check(hipGetLastError());
}

}  // namespace qk
