#pragma once
// Device code of the fault-tolerant batched FFT for CDNA4 (gfx950): the pass
// kernel, the correction kernel and their per-(element type, length)
// launchers.  Each (type, length) pair is instantiated in a translation unit
// of its own (tfft_inst.hip, compiled once per pair), so that the kernels
// build in parallel; tfft_kernels.hip dispatches to them.
//
//
// One launch per pass of the tiled FFT (TurboFFT Section IV-A.1).  A
// workgroup owns one checksum group at a time (Section IV-B.2, the
// threadblock-level two-sided checksum) and walks its members a tile of C
// signals at a time:
//   load   coalesced global loads of the next tile issued while the current
//          one is transformed (complex64: into registers; complex128: straight
//          into a second LDS buffer); on the loaded values the pre-transform
//          checksum c . x (fp64) is accumulated, weighted by 1 and by the
//          member's one-based index (Section III, Eq. (4)-(5));
//   stages Stockham radix-E butterflies held in registers (the thread-level
//          macro FFT, Section IV-A.2) with LDS transposes between stages;
//          stage twiddles come from an fp64-generated table rounded once;
//   store  post-transform checksum e . y in fp64 on the final registers, then
//          coalesced stores;
//   check  one workgroup reduction per group; a residual beyond tau is
//          recorded with the residual quotient that locates the member.
// Flagged groups are corrected afterwards by a separate launch (delayed,
// batched correction, Section III-B) that rebuilds the located member from
// the transform of the group's combined input, in fp64.  Template variants
// give the one-sided (per-signal) and thread-level (per-butterfly) schemes
// compared in Section V.
#include <type_traits>
#include <utility>

#include "tfft_internal.h"

namespace tfft {

// ------------------------------------------------------------- complex
template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cmulconj(cx<R> a, cx<R> b) {  // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

template <typename R>
struct vec2;
template <>
struct vec2<float> { using type = float2; };
template <>
struct vec2<double> { using type = double2; };

template <typename R>
__device__ __forceinline__ cx<R> ldg(const cx<R> *p) {
    typename vec2<R>::type v = *reinterpret_cast<const typename vec2<R>::type *>(p);
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stg(cx<R> *p, cx<R> a) {
    typename vec2<R>::type v;
    v.x = a.re;
    v.y = a.im;
    *reinterpret_cast<typename vec2<R>::type *>(p) = v;
}
// Signal data: read once and written once per pass (streaming).
template <typename R>
using nvec2 = R __attribute__((ext_vector_type(2)));

template <typename R>
__device__ __forceinline__ cx<R> ld_stream(const cx<R> *p) {
    if constexpr (TFFT_NT) {
        const nvec2<R> v = __builtin_nontemporal_load(reinterpret_cast<const nvec2<R> *>(p));
        return {v.x, v.y};
    } else {
        return ldg(p);
    }
}
template <typename R, bool NTS = true>
__device__ __forceinline__ void st_stream(cx<R> *p, cx<R> a) {
    if constexpr (TFFT_NT && NTS) {
        nvec2<R> v;
        v.x = a.re;
        v.y = a.im;
        __builtin_nontemporal_store(v, reinterpret_cast<nvec2<R> *>(p));
    } else {
        stg(p, a);
    }
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// ---------------------------------------------------- small DFT in registers
// Multiply by w_LEN^K = exp(-2 pi i K / LEN) for compile-time K < LEN/2,
// LEN <= 16; trivial factors cost no multiplication.
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kCos1_16 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kSin1_16 = 0.38268343236508977173;  // sin(pi/8)

template <typename R, int K, int LEN>
__device__ __forceinline__ cx<R> mul_wconst(cx<R> x) {
    constexpr int idx = (K * 16) / LEN;  // angle = 2 pi idx / 16
    if constexpr (idx == 0) {
        return x;
    } else if constexpr (idx == 4) {
        return {x.im, -x.re};
    } else if constexpr (idx == 2) {
        const R h = R(kSqrtHalf);
        return {h * (x.re + x.im), h * (x.im - x.re)};
    } else if constexpr (idx == 6) {
        const R h = R(kSqrtHalf);
        return {h * (x.im - x.re), -h * (x.re + x.im)};
    } else {
        constexpr double c = idx == 1 ? kCos1_16 : idx == 3 ? kSin1_16 : idx == 5 ? -kSin1_16 : -kCos1_16;
        constexpr double s = idx == 1 ? kSin1_16 : idx == 3 ? kCos1_16 : idx == 5 ? kCos1_16 : kSin1_16;
        return {x.re * R(c) + x.im * R(s), x.im * R(c) - x.re * R(s)};
    }
}

constexpr int bitrev_c(int v, int bits) { return bits == 0 ? 0 : ((v & 1) << (bits - 1)) | bitrev_c(v >> 1, bits - 1); }

// In-place length-RAD DFT (forward) of v[0..RAD): iterative radix-2
// decimation in time on bit-reversed registers, natural-order output.
template <typename R, int RAD>
__device__ __forceinline__ void dft_small(cx<R> *v) {
    if constexpr (RAD > 1) {
        constexpr int BITS = ilog2c(RAD);
        cx<R> a[RAD];
        static_for<0, RAD>([&](auto i) { a[i] = v[bitrev_c(i, BITS)]; });
        static_for<1, BITS + 1>([&](auto L) {
            constexpr int LEN = 1 << L;
            static_for<0, RAD / LEN>([&](auto blk) {
                static_for<0, LEN / 2>([&](auto k) {
                    constexpr int i0 = blk * LEN + k;
                    constexpr int i1 = i0 + LEN / 2;
                    const cx<R> t = mul_wconst<R, k, LEN>(a[i1]);
                    const cx<R> u = a[i0];
                    a[i0] = cadd(u, t);
                    a[i1] = csub(u, t);
                });
            });
        });
        static_for<0, RAD>([&](auto i) { v[i] = a[i]; });
    }
}

// ------------------------------------------------------ per-stage constants
template <int M, int E>
struct Stages {
    static constexpr int count = n_stages(M, E);
    static constexpr int T = M / E;
    static constexpr int radix(int s) { return stage_radix(M, E, s); }
    static constexpr int ns(int s) { return stage_ns(M, E, s); }
    static constexpr int nb(int s) { return E / stage_radix(M, E, s); }
    // twiddle registers of stages 1..s-1
    static constexpr int tw_off(int s) { return s <= 1 ? 0 : tw_off(s - 1) + nb(s - 1) * (radix(s - 1) - 1); }
    static constexpr int tw_count() { return tw_off(count) > 0 ? tw_off(count) : 1; }
};

// ----------------------------------------------------------- addressing
// Where member b of group g lives.  Offsets inside one signal are below
// N <= 2^24, so the in-signal part is 32-bit.
struct MemberLoc {
    int64_t in_off, out_off;
    uint32_t in_stride, out_stride;
    int64_t tw_i;  // STRIDED: position inside the stride (twiddle exponent factor)
    bool valid;
};

template <int M, int KIND, int C>
__device__ __forceinline__ MemberLoc member_loc(const PassArgs &a, int64_t g, int b) {
    MemberLoc L;
    if constexpr (KIND == KIND_ROWS) {
        const int64_t s = g * a.G + b;
        L.valid = s < a.batch;
        const int64_t sc = L.valid ? s : 0;
        L.in_off = a.in_sig ? a.in_sig[sc] : s * M;
        L.out_off = a.out_sig ? a.out_sig[sc] : s * M;
        L.in_stride = 1;
        L.out_stride = 1;
        L.tw_i = 0;
    } else {
        // n_strips and O are powers of two: shifts and masks (TFFT_MEMBER_SHIFT)
        // or divisions
        const int64_t strip = TFFT_MEMBER_SHIFT ? (g & (a.n_strips - 1)) : g % a.n_strips;
        const int64_t u = (TFFT_MEMBER_SHIFT ? (g >> a.ns_log2) : g / a.n_strips) * a.rb + b / C;  // outer unit
        const int64_t r = strip * C + b % C;                 // sub-signal inside the unit
        L.valid = u < a.n_outer;
        if constexpr (KIND == KIND_STRIDED) {
            const int64_t beta = L.valid ? (TFFT_MEMBER_SHIFT ? (u >> a.o_log2) : u / a.O) : 0;
            const int64_t o = TFFT_MEMBER_SHIFT ? (u & (a.O - 1)) : u % a.O;
            L.in_off = (a.in_sig ? a.in_sig[beta] : beta * a.n) + o * a.L + r;
            L.out_off = (a.out_sig ? a.out_sig[beta] : beta * a.n) + o * a.L + r;
            L.in_stride = (uint32_t)a.S;
            L.out_stride = (uint32_t)a.S;
            L.tw_i = r;
        } else {
            const int64_t o = (r & (a.m1 - 1)) * a.m2 + (r >> a.m1_log2);
            const int64_t beta = L.valid ? u : 0;
            L.in_off = (a.in_sig ? a.in_sig[beta] : u * a.n) + o * M;
            L.out_off = (a.out_sig ? a.out_sig[beta] : u * a.n) + r;
            L.in_stride = 1;
            L.out_stride = (uint32_t)a.rows;
            L.tw_i = 0;
        }
    }
    return L;
}

// Members of group g that exist (a prefix 0..count-1 of the G members: the
// last group of a batch, or of the outer units, may be partial).
template <int KIND, int C>
__device__ __forceinline__ int group_members(const PassArgs &a, int64_t g) {
    if constexpr (KIND == KIND_ROWS) {
        const int64_t left = a.batch - g * a.G;
        return left < a.G ? (int)left : a.G;
    } else {
        const int64_t left = a.n_outer - (g / a.n_strips) * a.rb;
        return C * (left < a.rb ? (int)left : a.rb);
    }
}

// LDS element index of position `pos` of tile slot `slot`, XOR-swizzled
// inside each 256-byte bank row so that the Stockham scatter writes, the
// strided reads and the transposed-store re-map hit distinct banks.  The
// swizzle is a unit-triangular map over GF(2) of the low bits: a bijection
// on every power-of-two tile.
template <typename R, int M, int C, int KIND>
__device__ __forceinline__ int lds_index(int slot, int pos) {
    constexpr int RE = 256 / (2 * (int)sizeof(R));  // elements per bank row
    if constexpr (KIND == KIND_STRIDED) {
        const int L = pos * C + slot;
        return L ^ ((L >> 3) & (RE - 1));
    } else {
        const int L = slot * M + pos;
        return L ^ (((L >> 3) ^ (L >> 7)) & (RE - 1));
    }
}

// w_N^t from the two-level fp64 table.
__device__ __forceinline__ cx<double> itw(const PassArgs &a, int64_t t) {
    const int64_t mask = (int64_t(1) << a.itw_bits) - 1;
    const cx<double> lo = ldg(reinterpret_cast<const cx<double> *>(a.itw_lo) + (t & mask));
    const cx<double> hi = ldg(reinterpret_cast<const cx<double> *>(a.itw_hi) + (t >> a.itw_bits));
    return cmul(lo, hi);
}

// Fault hook (test instrument): the register of this thread that a fault of
// the group hits at `stage`, or m = -1.  Returned by value so that the
// register array of the caller is never address-taken (it would be placed in
// scratch memory).
struct FaultHit {
    int m;                  // register index, -1 = none
    double dre, dim;        // additive part
    unsigned long long fre, fim;  // bit masks to flip in re / im
};

__device__ __forceinline__ FaultHit find_fault(const DevFault *F, int fh, int stage, int b, int j) {
    FaultHit h{-1, 0.0, 0.0, 0ull, 0ull};
    for (int f = fh; f >= 0; f = F[f].next) {
        DevFault x = F[f];
        // every field in registers before any is tested: a load left in
        // flight on a path that never reads it would make the code after
        // the fault hook wait for the whole vector-memory queue (the LDS-DMA
        // prefetch in flight included) before reusing its register
        asm volatile("" : "+v"(x.member), "+v"(x.stage), "+v"(x.j), "+v"(x.m), "+v"(x.mode), "+v"(x.bit),
                     "+v"(x.dre), "+v"(x.dim));
        if (x.stage == stage && x.member == b && x.j == j) {
            if (h.m < 0 || h.m == x.m) {
                h.m = x.m;
                if (x.mode == 0) {
                    h.dre += x.dre;
                    h.dim += x.dim;
                } else if (x.mode == 1) {
                    h.fre ^= 1ull << x.bit;
                } else {
                    h.fim ^= 1ull << x.bit;
                }
            }
        }
    }
    return h;
}

__device__ __forceinline__ float flip_bits(float v, unsigned long long mask) {
    return __uint_as_float(__float_as_uint(v) ^ (unsigned int)mask);
}
__device__ __forceinline__ double flip_bits(double v, unsigned long long mask) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)mask);
}

template <typename R, int E>
__device__ __forceinline__ void apply_hit(cx<R> (&d)[E], const FaultHit &h);

template <typename R, int E>
__device__ __forceinline__ void apply_faults(cx<R> (&d)[E], const DevFault *F, int fh, int stage, int b, int j) {
    apply_hit<R, E>(d, find_fault(F, fh, stage, b, j));
}

// The usual case of one fault in the group: its spec is read once per group
// (f0) and each stage only compares, instead of walking the list in global
// memory after every stage.
__device__ __forceinline__ FaultHit fault_hit_g(const DevFault &f0, bool multi, const DevFault *F, int fh, int stage,
                                               int b, int j) {
    if (multi) return find_fault(F, fh, stage, b, j);
    FaultHit h{-1, 0.0, 0.0, 0ull, 0ull};
    if (f0.stage == stage && f0.member == b && f0.j == j) {
        h.m = f0.m;
        if (f0.mode == 0) {
            h.dre = f0.dre;
            h.dim = f0.dim;
        } else if (f0.mode == 1) {
            h.fre = 1ull << f0.bit;
        } else {
            h.fim = 1ull << f0.bit;
        }
    }
    return h;
}

template <typename R, int E>
__device__ __forceinline__ void apply_faults_g(cx<R> (&d)[E], const DevFault &f0, bool multi, const DevFault *F,
                                               int fh, int stage, int b, int j) {
    apply_hit<R, E>(d, fault_hit_g(f0, multi, F, fh, stage, b, j));
}

// The fault of h applied to register m's value v (a select, no indexing).
template <typename R>
__device__ __forceinline__ cx<R> hit_one(cx<R> v, const FaultHit &h, int m) {
    const bool hit = m == h.m;
    v.re = flip_bits(v.re + (hit ? R(h.dre) : R(0)), hit ? h.fre : 0ull);
    v.im = flip_bits(v.im + (hit ? R(h.dim) : R(0)), hit ? h.fim : 0ull);
    return v;
}

template <typename R, int E>
__device__ __forceinline__ void apply_hit(cx<R> (&d)[E], const FaultHit &h) {
    // Every register takes an addend and a flip mask that are zero except at
    // h.m: written as an add of a selected value and an xor with a selected
    // mask (not a conditional update) so the compiler cannot turn it into an
    // indexed store that would demote d[] to scratch memory.
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const bool hit = m == h.m;
        d[m].re = flip_bits(d[m].re + (hit ? R(h.dre) : R(0)), hit ? h.fre : 0ull);
        d[m].im = flip_bits(d[m].im + (hit ? R(h.dim) : R(0)), hit ? h.fim : 0ull);
    }
}

constexpr double kW3r = -0.5;
static __device__ const int32_t kNoFault = -1;
constexpr double kW3i = -0.86602540378443864676;  // w_3 = exp(-2 pi i / 3)

__device__ __forceinline__ double wave_sum(double v, int width) {
    for (int off = width / 2; off > 0; off /= 2) v += __shfl_xor(v, off, width);
    return v;
}

// DPP moves of a 64-bit value (two 32-bit halves); lanes outside row_mask
// read 0.  With every row enabled each lane has a valid source, so the move
// needs no zeroed destination first (one instruction per half, not two).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_b32(int v) {
    if constexpr (ROWMASK == 0xF) return __builtin_amdgcn_mov_dpp(v, CTRL, ROWMASK, 0xF, false);
    else return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_b32<CTRL, ROWMASK>((int)(b & 0xffffffffll));
    const int hi = dpp_b32<CTRL, ROWMASK>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp32(float v) {
    return __int_as_float(dpp_b32<CTRL, ROWMASK>(__float_as_int(v)));
}

// Sum over a full 64-lane wavefront with DPP lane moves (no LDS traffic):
// butterflies inside quads and rows of 16, then the row broadcasts; the total
// ends in lane 63.
template <typename T, typename F>
__device__ __forceinline__ T wave_sum_dpp(T v, F mv) {
    v += mv.template operator()<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += mv.template operator()<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += mv.template operator()<0x124, 0xF>(v);  // row_ror:4
    v += mv.template operator()<0x128, 0xF>(v);  // row_ror:8
    v += mv.template operator()<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v += mv.template operator()<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
    return v;
}
struct Dpp64 {
    template <int C, int RM>
    __device__ __forceinline__ double operator()(double v) const { return dpp64<C, RM>(v); }
};
struct Dpp32 {
    template <int C, int RM>
    __device__ __forceinline__ float operator()(float v) const { return dpp32<C, RM>(v); }
};

// ------------------------------------------------------------- pass kernel
// cos(15 degrees * i), i = 0..23: the angles 2 pi t / (3 RAD) of the
// butterfly encodings for RAD in {2, 4, 8} are multiples of 15 degrees.
constexpr double kCos15[24] = {1.0, 0.96592582628906831, 0.86602540378443865, 0.70710678118654752, 0.5,
                               0.25881904510252076, 0.0, -0.25881904510252076, -0.5, -0.70710678118654752,
                               -0.86602540378443865, -0.96592582628906831, -1.0, -0.96592582628906831,
                               -0.86602540378443865, -0.70710678118654752, -0.5, -0.25881904510252076, 0.0,
                               0.25881904510252076, 0.5, 0.70710678118654752, 0.86602540378443865,
                               0.96592582628906831};
template <int RAD>
constexpr double kCos3R(int t) { return kCos15[(t * (8 / RAD)) % 24]; }
template <int RAD>
constexpr double kSin3R(int t) { return kCos15[(t * (8 / RAD) + 18) % 24]; }

// Two-sided check of one radix-RAD butterfly inside its thread (FT_THREAD).
// The butterfly maps its (twiddled) inputs v to y = W_RAD v.  Transform
// encodings e_k = w_3^k and (k+1) e_k on the outputs are compared with their
// precomputed images c1 = W^T e and c2 = W^T ((k+1) e) applied to the inputs:
// d1 = e.y - c1.v, d2 = ((k+1) e).y - c2.v.  A single wrong output y_k gives
// d2 / d1 = k + 1; the butterfly is then recomputed from v (in CORRECT mode)
// and the event recorded.  binary64 throughout; tau as for a group, with M =
// RAD and S the energy of v.
template <int RAD>
struct ButterflyEnc {
    static_assert(RAD == 2 || RAD == 4 || RAD == 8, "butterfly encodings use a 15-degree table: radix 2, 4 or 8");
    double c1r[RAD], c1i[RAD], c2r[RAD], c2i[RAD];
    constexpr ButterflyEnc() : c1r(), c1i(), c2r(), c2i() {
        for (int q = 0; q < RAD; ++q) {
            double ar = 0, ai = 0, br = 0, bi = 0;
            for (int k = 0; k < RAD; ++k) {
                // e_k w_RAD^{kq} = exp(-2 pi i (k/3 + kq/RAD)): angle index over 3 RAD
                const int t = (k * RAD + 3 * k * q) % (3 * RAD);
                const double cr = kCos3R<RAD>(t), ci = -kSin3R<RAD>(t);
                ar += cr;
                ai += ci;
                br += (k + 1) * cr;
                bi += (k + 1) * ci;
            }
            c1r[q] = ar;
            c1i[q] = ai;
            c2r[q] = br;
            c2i[q] = bi;
        }
    }
};

template <typename R, int RAD, int NB, int P, int E>
__device__ __forceinline__ void thread_check(cx<R> (&d)[E], const cx<R> (&vin)[E], const PassArgs &a, int64_t g,
                                             int b, int s) {
    constexpr ButterflyEnc<RAD> enc{};
    double l1r = 0, l1i = 0, l2r = 0, l2i = 0, r1r = 0, r1i = 0, r2r = 0, r2i = 0, S = 0;
#pragma unroll
    for (int q = 0; q < RAD; ++q) {
        const double vr = double(vin[P + q * NB].re), vi = double(vin[P + q * NB].im);
        l1r += enc.c1r[q] * vr - enc.c1i[q] * vi;
        l1i += enc.c1r[q] * vi + enc.c1i[q] * vr;
        l2r += enc.c2r[q] * vr - enc.c2i[q] * vi;
        l2i += enc.c2r[q] * vi + enc.c2i[q] * vr;
        S += vr * vr + vi * vi;
        // e_q = w_3^(q mod 3)
        const double yr = double(d[P + q * NB].re), yi = double(d[P + q * NB].im);
        const int cls = q % 3;
        const double er = cls == 0 ? 1.0 : kW3r, ei = cls == 0 ? 0.0 : (cls == 1 ? kW3i : -kW3i);
        const double tr = er * yr - ei * yi, ti = er * yi + ei * yr;
        r1r += tr;
        r1i += ti;
        r2r += (q + 1) * tr;
        r2i += (q + 1) * ti;
    }
    const double d1r = r1r - l1r, d1i = r1i - l1i, d2r = r2r - l2r, d2i = r2i - l2i;
    constexpr double kLog = RAD == 2 ? 1.0 : (RAD == 4 ? 1.4142135623730951 : 1.7320508075688772);
    const double tau = a.kappa_u * kLog * sqrt(double(RAD) * S);
    if (!(sqrt(d1r * d1r + d1i * d1i) <= tau)) {
        const double den = d1r * d1r + d1i * d1i;
        const double rhor = (d2r * d1r + d2i * d1i) / den, rhoi = (d2i * d1r - d2r * d1i) / den;
        if (a.fix) {
            cx<R> v[RAD];
#pragma unroll
            for (int q = 0; q < RAD; ++q) v[q] = vin[P + q * NB];
            dft_small<R, RAD>(v);
#pragma unroll
            for (int q = 0; q < RAD; ++q) d[P + q * NB] = v[q];
            atomicAdd(&a.rep->corrected, 1ULL);
        }
        const unsigned long long slot = atomicAdd(&a.rep->n_flag, 1ULL);
        if ((int64_t)slot < a.rec_cap) {
            DevRecord rc;
            rc.group = a.g_base + g;
            rc.pass = a.pass;
            rc.task = a.task;
            rc.action = a.fix ? 2 : 1;  // corrected in registers, or detected
            rc.member = b;
            rc.method = 3;  // located inside the thread's butterfly
            rc.d1r = d1r;
            rc.d1i = d1i;
            rc.d2r = d2r;
            rc.d2i = d2i;
            rc.tau = tau;
            rc.s = double(s);
            a.recs[slot] = rc;
        }
        (void)rhor;
        (void)rhoi;
    }
}

// FT selects the checksum scheme: FT_NONE (no checking), FT_BLOCK (two-sided,
// one residual pair per group of G signals, reduced over the workgroup),
// FT_SIGNAL (one-sided: one residual per signal, reduced over the signal's
// threads; a flagged signal is recomputed) or FT_THREAD (two-sided checks of
// every radix butterfly inside the thread that computes it, corrected in
// registers).  In one-pass plans FT_SIGNAL makes every signal a group of its
// own (tiles of C groups); in the passes of multi-pass plans it keeps the
// tiles of FT_BLOCK and checks every sub-signal of a tile separately.
#if TFFT_WAVES_PER_EU > 0
#define TFFT_PASS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(TFFT_WAVES_PER_EU)))
#else
#define TFFT_PASS_OCCUPANCY
#endif
// Compile-time shape of a pass kernel.  NTHR = 0: the tile of the dense
// configuration (cfg_C); NTHR > 0: tiles of NTHR / T signals, so that every
// variant fills a workgroup of NTHR threads (the persistent ragged kernel).
template <typename R, int M, int KIND, int FT, int NTHR = 0>
struct PassCfg {
    static constexpr int FP64 = sizeof(R) == 8;
    static constexpr bool BLK = FT == FT_BLOCK, SIG = FT == FT_SIGNAL, THR = FT == FT_THREAD;
    static constexpr bool PF_FENCE = cfg_pf_fence(FP64, M, KIND) != 0;
    static constexpr int E = cfg_E(FP64, M, KIND);
    static constexpr int T = M / E;
    static constexpr int C = NTHR > 0 ? (NTHR / T > 0 ? NTHR / T : 1) : cfg_C(FP64, M, KIND);
    static constexpr int NT = C * T;
    // Non-temporal stores, except for tiles whose rows are narrower than a
    // 128-byte line: there the two halves of a line come from different
    // workgroups and must meet in L2 (measured: streaming them wrote up to
    // 26% more bytes than the output holds).
    static constexpr bool NT_ST = KIND == KIND_ROWS || (C * int(sizeof(R)) * 2 >= TFFT_NT_MIN_ROW &&
                                                        (KIND == KIND_LAST || TFFT_NT_STRIDED_ST));
    static constexpr bool ENC = BLK || SIG;          // input and output encodings
    static constexpr bool SIGR = SIG && KIND == KIND_ROWS;  // one-sided, tiles of one-signal groups
    static constexpr bool SIGM = SIG && KIND != KIND_ROWS;  // one-sided, per sub-signal of block tiles
    static constexpr int NSTAGE = n_stages(M, E);
    static constexpr int WAVES = (NT + 63) / 64;
    static constexpr int WIDTH = NT < 64 ? NT : 64;
    // group sums reduced through LDS (see the end of a group)
    static constexpr bool LDS_RED = TFFT_LDS_RED && NT % 64 == 0 && NT > 64 &&
                                    C * M * int(sizeof(R)) * 2 >= 5 * NT * int(sizeof(double));
    // block scheme: a group's decision deferred into the next group, which
    // needs at least one workgroup barrier inside every group
    static constexpr bool RED_DEFER = TFFT_RED_DEFER && BLK && !LDS_RED && NT % 64 == 0 &&
                                      (NSTAGE >= 2 || KIND == KIND_LAST);
    static constexpr bool TWREG = cfg_twreg(FP64, M, KIND) != 0;
    static constexpr bool CREG = ENC && cfg_creg(FP64, M, KIND) != 0;
    // prefetch of the next tile straight into a second LDS buffer (16-byte
    // elements, whole wavefronts, both buffers within 128 KiB)
    static constexpr bool LDSPF = FP64 && (TFFT_LDSPF64 == 2 || (TFFT_LDSPF64 == 1 && KIND == KIND_ROWS)) &&
                                  M >= TFFT_LDSPF64_MIN && C * M * 16 * 2 <= 131072 && NT % 64 == 0;
    static constexpr bool TWLDS = !TWREG && (LDSPF || cfg_twlds(FP64, M, KIND)) && M >= 8;
    static constexpr bool PREFETCH = !LDSPF && cfg_prefetch(FP64, M, KIND) != 0;
    static constexpr bool DEFER = cfg_defer(FP64, M, KIND) && (LDSPF || (PREFETCH && PF_FENCE));
};

// The LDS of one pass kernel variant: the exchange tile, the group-sum
// slots, the twiddle octant, the prefetch buffer, the one-sided partial sums
// and the group's first fault.
template <typename R, int M, int KIND, int FT, int NTHR = 0>
struct PassShared {
    using Cf = PassCfg<R, M, KIND, FT, NTHR>;
    alignas(16) cx<R> lds[Cf::C * M];
    double red[Cf::WAVES][5];
    double redg[Cf::RED_DEFER ? 2 : 1][Cf::RED_DEFER ? Cf::WAVES : 1][5];
    cx<R> twl[Cf::TWLDS ? M / 8 + 1 : 1];
    double redm[Cf::SIGM && KIND == KIND_STRIDED ? Cf::WAVES : 1][Cf::SIGM && KIND == KIND_STRIDED ? Cf::C : 1][3];
    DevFault f0;
};

// The LDS-DMA prefetch buffer (16-byte aligned: the DMA writes 16 bytes per
// lane) is an LDS variable of its own, not a member of PassShared: accesses
// to distinct LDS variables carry distinct alias scopes, so the compiler
// knows that the stage exchanges through `lds` do not touch the buffer the
// DMA in flight is writing, and does not wait for the DMA before them.
template <typename R, int M, int KIND, int FT, int NTHR = 0>
constexpr int pass_nbuf_elems() {
    using Cf = PassCfg<R, M, KIND, FT, NTHR>;
    return Cf::LDSPF ? Cf::C * M : 1;
}

// Workgroup barrier for LDS traffic only: the wavefront's LDS operations
// complete, then s_barrier; the memory clobber keeps the compiler from moving
// memory operations across it.  __syncthreads also waits for the
// wavefront's LDS-DMA loads in flight (its release fence covers LDS written
// by DMA), which would end the next tile's prefetch at the first exchange.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Wait for every vector-memory operation of the wavefront (vmcnt(0)) with
// the compiler's own wait instruction, between two compiler barriers for
// memory operations.  Written as inline asm the wait is opaque to the
// compiler's wait-count insertion, which then still counts the older loads
// as outstanding and waits for them again later, after newer stores (and so
// for those stores too).
__device__ __forceinline__ void vm_wait_all() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt 0; expcnt, lgkmcnt not waited
    asm volatile("" ::: "memory");
}

// Optional per-call hooks of pass_body: `slots` collects the record slots the
// call appends (the persistent kernel corrects them before it releases the
// item), at most `slot_cap` of them, counted in *n_slots.
struct PassHooks {
    int64_t *slots;
    int *n_slots;
    int slot_cap;
};

// The groups g_first, g_first + g_step, ... (< g_end) of one pass, processed
// by one workgroup of PassCfg::NT threads with the LDS of `sh`.
template <typename R, int M, int KIND, int FT, int NTHR>
__device__ __forceinline__ void pass_body(const PassArgs &a, PassShared<R, M, KIND, FT, NTHR> &sh, cx<R> *nbuf,
                                          int64_t g_first, int64_t g_end, int64_t g_step, const PassHooks &hk) {
    using Cf = PassCfg<R, M, KIND, FT, NTHR>;
    constexpr int FP64 = Cf::FP64;
    constexpr bool BLK = Cf::BLK, SIG = Cf::SIG, THR = Cf::THR;
    constexpr bool PF_FENCE = Cf::PF_FENCE;
    constexpr bool NT_ST = Cf::NT_ST;
    constexpr bool ENC = Cf::ENC;
    constexpr bool SIGR = Cf::SIGR;
    constexpr bool SIGM = Cf::SIGM;
    constexpr int E = Cf::E;
    constexpr int T = Cf::T;
    constexpr int C = Cf::C;
    constexpr int NT = Cf::NT;
    using St = Stages<M, E>;
    constexpr int NSTAGE = St::count;
    constexpr int WAVES = Cf::WAVES;
    constexpr int WIDTH = Cf::WIDTH;
    constexpr bool LDS_RED = Cf::LDS_RED;
    constexpr bool RED_DEFER = Cf::RED_DEFER;

    auto &lds = sh.lds;
    auto &red = sh.red;
    auto &redg = sh.redg;
    // the barriers of the pass: LDS-only where a DMA prefetch may be in flight
    auto tile_sync = [] {
        if constexpr (Cf::LDSPF) lds_barrier();
        else __syncthreads();
    };

    int tid = threadIdx.x;
    // persistent kernel: an opaque copy per call, so that what derives from
    // the lane index is computed per item, not hoisted out of the item loop
    // (every variant's lane constants would stay live across the whole loop)
    if constexpr (NTHR > 0) asm volatile("" : "+v"(tid));
    int c, j;
    if constexpr (KIND == KIND_STRIDED) {
        c = tid % C;
        j = tid / C;
    } else {
        c = tid / T;
        j = tid % T;
    }
    const cx<R> *in = reinterpret_cast<const cx<R> *>(a.in);
    cx<R> *out = reinterpret_cast<cx<R> *>(a.out);

    auto lidx = [](int slot, int pos) -> int { return lds_index<R, M, C, KIND>(slot, pos); };

    // Stage twiddles w_{NS*RAD}^{(i mod NS) q} (from the table of w_M^t) and
    // the pre-transform checksum vector at positions j + T m: either kept in
    // registers for all signals of the workgroup or re-read per signal.
    constexpr bool TWREG = Cf::TWREG;
    constexpr bool CREG = Cf::CREG;
    const cx<R> *stw = reinterpret_cast<const cx<R> *>(a.stw);
    const cx<double> *cv = reinterpret_cast<const cx<double> *>(a.cvec);
    // With the LDS prefetch, stage twiddles come from an LDS copy of the
    // first octant, w_M^t for t <= M/8, and the exact symmetries of the
    // table (the host builds it from the same octant): no global load in the
    // transform, whose wait would also wait for the prefetch.
    constexpr bool TWLDS = Cf::TWLDS;
    auto &twl = sh.twl;
    if constexpr (TWLDS) {
        for (int t = tid; t <= M / 8; t += NT) twl[t] = ldg(stw + t);
        tile_sync();
    }
    auto tw_oct = [&](int t) -> cx<R> {
        constexpr int M4 = M / 4, M8 = M / 8;
        const int qd = t / M4, r = t % M4;
        const cx<R> v = twl[r <= M8 ? r : M4 - r];
        // w^r for r > M/8 is (-Im, -Re) of w^(M/4 - r)
        const R a = r <= M8 ? v.re : -v.im, b = r <= M8 ? v.im : -v.re;
        // times (-i)^qd
        const R re = qd == 0 ? a : (qd == 1 ? b : (qd == 2 ? -a : -b));
        const R im = qd == 0 ? b : (qd == 1 ? -a : (qd == 2 ? -b : a));
        return cx<R>{re, im};
    };
    auto stage_tw = [&](auto S, auto p, auto q) -> cx<R> {
        constexpr int s = S;
        constexpr int RAD = St::radix(s), NS = St::ns(s);
        const int i = j + p * T;
        const int t = ((i % NS) * q) * (M / (NS * RAD));
        if constexpr (TWLDS) return tw_oct(t);
        else return ldg(stw + t);
    };
    cx<R> tw[TWREG ? St::tw_count() : 1];
    if constexpr (TWREG) {
        static_for<1, NSTAGE>([&](auto S) {
            constexpr int s = S;
            constexpr int RAD = St::radix(s), NB = St::nb(s);
            static_for<0, NB>([&](auto p) {
                static_for<1, RAD>([&](auto q) { tw[St::tw_off(s) + p * (RAD - 1) + (q - 1)] = stage_tw(S, p, q); });
            });
        });
    }
    cx<double> cc[CREG ? E : 1];
    if constexpr (CREG) {
#pragma unroll
        for (int m = 0; m < E; ++m) cc[m] = ldg(cv + j + T * m);
    }
    // e_k = w_3^(k mod 3) with k = j + T m: class of register m, rotated by j
    const int jr = j % 3;
    const double rotr = jr == 0 ? 1.0 : kW3r;
    const double roti = jr == 0 ? 0.0 : (jr == 1 ? kW3i : -kW3i);

    // FT_SIGNAL: a tile of C signals per iteration, each its own group (G = 1)
    const int rounds = SIGR ? 1 : a.G / C;
    const int64_t n_iter = g_end;
    auto mloc = [&](int64_t gg, int rr) -> MemberLoc {
        if constexpr (SIGR) return member_loc<M, KIND, C>(a, gg * C + c, 0);
        else return member_loc<M, KIND, C>(a, gg, rr * C + c);
    };
    // Software pipeline: the loads of the next tile (next round, or round 0 of
    // this workgroup's next group) are issued before the current tile is
    // transformed, so every wavefront keeps two tiles of HBM reads in flight.
    cx<R> nx[E];
    bool nx_ok = false;
    auto load_tile = [&](int64_t gg, int rr) {
        const MemberLoc Ln = mloc(gg, rr);
        nx_ok = gg < n_iter && Ln.valid;
        if constexpr (PF_FENCE) {
            // branch-free: a missing member re-reads element 0 and is zeroed
            // when consumed, so the compiler's count of outstanding loads
            // stays exact across the loop (no join of two load states)
            const cx<R> *s = in + (nx_ok ? Ln.in_off : 0);
            const uint32_t st = nx_ok ? Ln.in_stride : 0u;
            const uint32_t j0 = nx_ok ? (uint32_t)j : 0u;
#pragma unroll
            for (int m = 0; m < E; ++m) nx[m] = ld_stream(s + (j0 + (uint32_t)(T * m)) * st);
        } else if (nx_ok) {
            const cx<R> *s = in + Ln.in_off;
#pragma unroll
            for (int m = 0; m < E; ++m) nx[m] = ld_stream(s + (uint32_t)(j + T * m) * Ln.in_stride);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) nx[m] = cx<R>{R(0), R(0)};
        }
    };
    // Asynchronous prefetch into LDS: the next tile's elements go straight
    // from HBM into a second LDS buffer (global_load_lds_dwordx4, no VGPRs
    // held) while the current tile is transformed.  Every thread prefetches
    // its own E elements of its own member; the instruction writes lane l of
    // a wavefront to slot base + l, so element m of thread tid goes to slot
    // m NT + tid, and a thread reads back only what its own lane wrote.
    constexpr bool LDSPF = Cf::LDSPF;
    constexpr bool PREFETCH = Cf::PREFETCH;
    auto nslot = [&](int m) -> int { return tid + NT * m; };
    auto dma_tile = [&](int64_t gg, int rr) {
        if constexpr (LDSPF) {
            static_assert(NT % 64 == 0 && sizeof(cx<R>) == 16, "LDS prefetch: 16-byte elements, full wavefronts");
            const MemberLoc Ln = mloc(gg, rr);
            // A member's offset may come from a table load (ragged plans).
            // Resolve it here, on every path: a load still pending where the
            // DMA is skipped would make the compiler wait for the whole
            // vector-memory queue, the DMA just issued included, at the
            // transform's first use of the register.
            int64_t in_off = Ln.in_off;
            asm volatile("" : "+v"(in_off));
            if (gg < n_iter && Ln.valid) {
                const cx<R> *src = in + in_off;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int base = nslot(m) - (tid & 63);  // wavefront-uniform
                    __builtin_amdgcn_global_load_lds((const void *)(src + (uint32_t)(j + T * m) * Ln.in_stride),
                                                     (__attribute__((address_space(3))) void *)(nbuf + base), 16,
                                                     0, 0);
                }
            }
        }
    };
    if constexpr (PREFETCH) load_tile(g_first, 0);
    if constexpr (LDSPF) dma_tile(g_first, 0);
    // Deferred stores (LDS-prefetching row tiles): a tile's outputs stay in
    // registers and are stored right after the next tile's prefetch has been
    // waited for, so that the wait (which also counts stores) never waits
    // for stores issued just before it.
    constexpr bool DEFER = Cf::DEFER;
    cx<R> ps[DEFER ? E : 1];
    cx<R> *pdst = out;     // first element of the pending stores
    uint32_t pstr = 1;     // their stride
    bool pend = false;
    auto flush = [&]() {
        if constexpr (DEFER) {
            if (pend) {
#pragma unroll
                for (int m = 0; m < E; ++m) st_stream<R, NT_ST>(pdst + (uint32_t)(T * m) * pstr, ps[m]);
            }
            pend = false;
        }
    };
    // One-sided check of each member (signal or sub-signal) of a tile: sum
    // the member's residual and energy over its threads, test it against its
    // own threshold and record it (method: 1 for a one-signal group, 4 for a
    // sub-signal of a block tile, which the correction recomputes alone).
    auto &redm = sh.redm;
    auto member_check = [&](int64_t grp, int mem, bool valid, double d1r, double d1i, double ssum, int method) {
        double v[3] = {d1r, d1i, ssum};
        bool mine;  // this thread reports the member
        if constexpr (KIND == KIND_STRIDED) {
            // threads of member c are the lanes c + C k
            for (int off = C; off < 64; off <<= 1) {
#pragma unroll
                for (int q = 0; q < 3; ++q) v[q] += __shfl_xor(v[q], off, 64);
            }
            if constexpr (NT > 64) {
                if ((tid & 63) < C) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) redm[tid >> 6][tid & 63][q] = v[q];
                }
                tile_sync();
                if (tid < C) {
                    v[0] = v[1] = v[2] = 0.0;
                    for (int w = 0; w < WAVES; ++w)
#pragma unroll
                        for (int q = 0; q < 3; ++q) v[q] += redm[w][tid][q];
                }
            }
            mine = tid < C;
        } else {
            // threads of member c are the T consecutive threads c T + j
            if constexpr (T <= 64) {
#pragma unroll
                for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q], T);
            } else {
#pragma unroll
                for (int q = 0; q < 3; ++q) v[q] = wave_sum_dpp(v[q], Dpp64{});
                if ((tid & 63) == 63) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) red[tid >> 6][q] = v[q];
                }
                tile_sync();
                if (j == 0) {
                    v[0] = v[1] = v[2] = 0.0;
                    for (int w = c * (T / 64); w < (c + 1) * (T / 64); ++w)
                        for (int q = 0; q < 3; ++q) v[q] += red[w][q];
                }
            }
            mine = j == 0;
        }
        if (mine && valid) {
            const double tau = a.tau_coef * sqrt(v[2]);
            if (!(sqrt(v[0] * v[0] + v[1] * v[1]) <= tau)) {
                const unsigned long long slot = atomicAdd(&a.rep->n_flag, 1ULL);
                if ((int64_t)slot < a.rec_cap) {
                    DevRecord rc;
                    rc.group = a.g_base + grp;
                    rc.pass = a.pass;
                    rc.task = a.task;
                    rc.action = 1;  // detected
                    rc.member = mem;
                    rc.method = method;
                    rc.d1r = v[0];
                    rc.d1i = v[1];
                    rc.d2r = v[0];  // one weight: the quotient is 1
                    rc.d2i = v[1];
                    rc.tau = tau;
                    rc.s = v[2];
                    a.recs[slot] = rc;
                }
            }
        }
        if constexpr (NT > 64) tile_sync();
    };
    // a group's decision from its five sums (one thread)
    auto decide = [&](const double *t, int64_t g) {
        const double d1r = t[0], d1i = t[1], d2r = t[2], d2i = t[3], S = t[4];
        const double tau = a.tau_coef * sqrt(S);
        const double ad1 = sqrt(d1r * d1r + d1i * d1i);
        if (!(ad1 <= tau)) {
            const double den = d1r * d1r + d1i * d1i;
            const double rhor = (d2r * d1r + d2i * d1i) / den;
            const double rhoi = (d2i * d1r - d2r * d1i) / den;
            int jl = -1;
            if (isfinite(rhor) && isfinite(rhoi)) {
                // only members that exist: the last group of a batch may be partial
                const double fj = floor(rhor + 0.5);
                if (fj >= 1.0 && fj <= double(group_members<KIND, C>(a, g))) {
                    const double er = rhor - fj;
                    if (sqrt(er * er + rhoi * rhoi) <= 0.25) jl = int(fj) - 1;
                }
            }
            const unsigned long long slot = atomicAdd(&a.rep->n_flag, 1ULL);
            if (hk.slots && *hk.n_slots < hk.slot_cap) hk.slots[(*hk.n_slots)++] = (int64_t)slot;
            if ((int64_t)slot < a.rec_cap) {
                DevRecord rc;
                rc.group = a.g_base + g;
                rc.pass = a.pass;
                rc.task = a.task;
                rc.action = 1;  // detected
                rc.member = jl;
                rc.method = jl >= 0 ? 1 : 0;
                rc.d1r = d1r;
                rc.d1i = d1i;
                rc.d2r = d2r;
                rc.d2i = d2i;
                rc.tau = tau;
                rc.s = S;
                a.recs[slot] = rc;
            }
        }
    };
    int64_t g_prev = -1;  // RED_DEFER: the group whose decision is pending
    int it = 0;           // RED_DEFER: groups done by this workgroup
    for (int64_t g = g_first; g < n_iter; g += g_step) {
        const int64_t gsig = g * C + c;  // FT_SIGNAL: this thread's signal (= its group)
        // the fault lookup reads a table entry or a constant -1 (no branch)
        const int32_t *fhp;
        if constexpr (SIGR) fhp = (a.fault_head && gsig < a.n_groups) ? a.fault_head + a.g_base + gsig : &kNoFault;
        else fhp = a.fault_head ? a.fault_head + a.g_base + g : &kNoFault;
        const int fh = *fhp;
        // the group's first fault, staged in LDS once (fh is uniform outside
        // FT_SIGNAL, whose threads walk the list themselves)
        DevFault &f0 = sh.f0;
        bool fmulti = true;
        if constexpr (!SIGR) {
            if (fh >= 0) {
                tile_sync();
                if (tid == 0) f0 = a.faults[fh];
                tile_sync();
                fmulti = f0.next >= 0;
            }
        }
        double D1r = 0.0, D1i = 0.0, D2r = 0.0, D2i = 0.0;
        double Ssum = 0.0;  // energy of the group's inputs (binary64), for the threshold only
        for (int r = 0; r < rounds; ++r) {
            const int b = SIGR ? 0 : r * C + c;
            const MemberLoc L = mloc(g, r);
            // offsets inside one signal are below N <= 2^24: 32-bit arithmetic
            cx<R> *dst = out + L.out_off;
            const uint32_t ostr = (uint32_t)L.out_stride;
            cx<R> d[E];
            // checksum vector at this thread's positions (when not kept in
            // registers) and the inter-pass twiddle of this member (strided
            // passes): loaded before any prefetch is issued, so that waiting
            // for them never waits for the prefetch
            cx<double> cl[ENC && !CREG ? E : 1];
            if constexpr (ENC && !CREG) {
#pragma unroll
                for (int m = 0; m < E; ++m) cl[m] = ldg(cv + j + T * m);
            }
            cx<double> twA{1.0, 0.0}, twB{1.0, 0.0};
            if constexpr (KIND == KIND_STRIDED) {
                // w_L^{k i} = w_N^{k i N/L}; N is a power of two, so the
                // exponent is reduced mod N with a mask
                twA = itw(a, (int64_t(j) * L.tw_i * a.tw_scale) & (a.n - 1));
                twB = itw(a, (int64_t(T) * L.tw_i * a.tw_scale) & (a.n - 1));
            }
            if constexpr (LDSPF) {
                // this tile's DMA (issued one iteration earlier) has landed;
                // each thread reads only the slots its own lane filled
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                flush();
#pragma unroll
                for (int m = 0; m < E; ++m) d[m] = L.valid ? nbuf[nslot(m)] : cx<R>{R(0), R(0)};
                // (the next DMA is issued after the input encoding below, so
                // that the checksum vector's loads do not wait for it)
            } else if constexpr (PREFETCH) {
#pragma unroll
                for (int m = 0; m < E; ++m) d[m] = (!PF_FENCE || nx_ok) ? nx[m] : cx<R>{R(0), R(0)};
                if constexpr (PF_FENCE) {
                    // Materialise this tile's values before the next tile's
                    // loads are issued: the vector-memory counter cannot tell
                    // the two apart, so a load hoisted above this point would
                    // make the wait for this tile also wait for the next one.
#pragma unroll
                    for (int m = 0; m < E; ++m) asm volatile("" : "+v"(d[m].re), "+v"(d[m].im));
                    asm volatile("" ::: "memory");
                }
                flush();
                if (r + 1 < rounds) load_tile(g, r + 1);
                else load_tile(g + g_step, 0);
            } else {
                load_tile(g, r);
#pragma unroll
                for (int m = 0; m < E; ++m) d[m] = (!PF_FENCE || nx_ok) ? nx[m] : cx<R>{R(0), R(0)};
            }
            if constexpr (ENC) {
                double lr = 0.0, li = 0.0;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const double xr = double(d[m].re), xi = double(d[m].im);
                    cx<double> cm;
                    if constexpr (CREG) cm = cc[m];
                    else cm = cl[m];
                    // chained fused multiply-adds into the running sums (two
                    // operations per product pair, not a product, a fused
                    // product and an add)
                    lr = __builtin_fma(cm.re, xr, lr);
                    lr = __builtin_fma(-cm.im, xi, lr);
                    li = __builtin_fma(cm.re, xi, li);
                    li = __builtin_fma(cm.im, xr, li);
                    Ssum = __builtin_fma(xr, xr, Ssum);
                    Ssum = __builtin_fma(xi, xi, Ssum);
                }
                D1r -= lr;
                D1i -= li;
                if constexpr (BLK) {
                    const double w2 = double(b + 1);
                    D2r -= w2 * lr;
                    D2i -= w2 * li;
                }
                if constexpr (LDSPF) asm volatile("" : "+v"(D1r), "+v"(D1i), "+v"(Ssum));
            }
            if constexpr (LDSPF && KIND == KIND_STRIDED)
                asm volatile("" : "+v"(twA.re), "+v"(twA.im), "+v"(twB.re), "+v"(twB.im));
            if constexpr (LDSPF && !ENC) {
                // This tile's values read out of the DMA buffer before the next
                // DMA is issued into it (the input encoding does the same for
                // the checksummed tiles): with a read still pending at the
                // DMA, the compiler waits for the DMA itself before using it.
#pragma unroll
                for (int m = 0; m < E; ++m) asm volatile("" : "+v"(d[m].re), "+v"(d[m].im));
            }
            if constexpr (LDSPF) {
                // Nothing older than the next tile's DMA outstanding in the
                // compiler's count (the previous tile's deferred stores have
                // drained by now): an older store still counted would make
                // the first exchange after the DMA wait for the whole queue.
                vm_wait_all();
                if (r + 1 < rounds) dma_tile(g, r + 1);
                else dma_tile(g + g_step, 0);
            }
            if (a.conj_in) {
#pragma unroll
                for (int m = 0; m < E; ++m) d[m].im = -d[m].im;
            }

            static_for<0, NSTAGE>([&](auto S) {
                constexpr int s = S;
                constexpr int RAD = St::radix(s), NS = St::ns(s), NB = St::nb(s);
                if constexpr (s > 0) {
#pragma unroll
                    for (int m = 0; m < E; ++m) d[m] = lds[lidx(c, j + T * m)];
                    tile_sync();
                    static_for<0, NB>([&](auto p) {
                        static_for<1, RAD>([&](auto q) {
                            cx<R> w;
                            if constexpr (TWREG) w = tw[St::tw_off(s) + p * (RAD - 1) + (q - 1)];
                            else w = stage_tw(S, p, q);
                            d[p + q * NB] = cmul(d[p + q * NB], w);
                        });
                    });
                }
                cx<R> vin[THR ? E : 1];  // FT_THREAD: the butterflies' inputs
                if constexpr (THR) {
#pragma unroll
                    for (int m = 0; m < E; ++m) vin[m] = d[m];
                }
                static_for<0, NB>([&](auto p) {
                    cx<R> v[RAD];
                    static_for<0, RAD>([&](auto q) { v[q] = d[p + q * NB]; });
                    dft_small<R, RAD>(v);
                    static_for<0, RAD>([&](auto q) { d[p + q * NB] = v[q]; });
                });
                if (fh >= 0) {
                    apply_faults_g<R, E>(d, f0, fmulti, a.faults, fh, s, b, j);
                    // FT_THREAD has no output encoding: a fault on a final
                    // value lands on the last butterfly's output
                    if constexpr (THR && s == NSTAGE - 1) apply_faults_g<R, E>(d, f0, fmulti, a.faults, fh, -1, b, j);
                }
                if constexpr (THR) {
                    static_for<0, NB>([&](auto p) {
                        constexpr int pp = p;
                        thread_check<R, RAD, NB, pp>(d, vin, a, g, b, s);
                    });
                }
                if constexpr (s < NSTAGE - 1) {
                    static_for<0, NB>([&](auto p) {
                        const int i = j + p * T;
                        const int base = (i / NS) * NS * RAD + (i % NS);
                        static_for<0, RAD>([&](auto q) { lds[lidx(c, base + q * NS)] = d[p + q * NB]; });
                    });
                    tile_sync();
                }
            });

            // final values: register m holds output position k = j + T m.  In
            // order: the inter-pass twiddle (strided passes), conjugation and
            // scale, the fault hook's final-value fault, the output encoding.
            double Ar[3] = {0.0, 0.0, 0.0}, Ai[3] = {0.0, 0.0, 0.0};  // sums of e-class 0, 1, 2
            FaultHit hf{-1, 0.0, 0.0, 0ull, 0ull};
            if constexpr (!THR) {
                if (fh >= 0) hf = fault_hit_g(f0, fmulti, a.faults, fh, -1, b, j);
            }
            if constexpr (KIND == KIND_STRIDED) {
                // w_N^{k sub} = A B^m with A = w_N^{j sub}, B = w_N^{T sub}: the
                // recurrence in fp64 serves both the twiddle (rounded once to
                // the element type) and the output encoding, which uses
                // e' = e conj(applied twiddle) (applied = P forward, conj(P)
                // inverse) so that the twiddle product is inside the check
                const double psg = a.conj_out ? -1.0 : 1.0;
                const bool scl = a.out_scale != 1.0;
                const R sc = R(a.out_scale);
                auto epilogue = [&](auto faulty) {
                    cx<double> P = twA;
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        cx<R> v = cmul(d[m], cx<R>{R(P.re), R(P.im)});
                        if (a.conj_out) v.im = -v.im;
                        if (scl) {
                            v.re *= sc;
                            v.im *= sc;
                        }
                        if constexpr (decltype(faulty)::value) v = hit_one(v, hf, m);
                        d[m] = v;
                        if constexpr (ENC) {
                            const int cls = ((T % 3) * m) % 3;
                            const double vr = double(v.re), vi = double(v.im);
                            const double pr = P.re, pi = psg * P.im;
                            Ar[cls] = __builtin_fma(vr, pr, Ar[cls]);
                            Ar[cls] = __builtin_fma(vi, pi, Ar[cls]);
                            Ai[cls] = __builtin_fma(vi, pr, Ai[cls]);
                            Ai[cls] = __builtin_fma(-vr, pi, Ai[cls]);
                        }
                        if (m + 1 < E) P = cmul(P, twB);
                    }
                };
                // the fault hook costs nothing unless the group has a fault
                if (!THR && fh >= 0) epilogue(std::true_type{});
                else epilogue(std::false_type{});
            } else {
                if (a.conj_out) {
#pragma unroll
                    for (int m = 0; m < E; ++m) d[m].im = -d[m].im;
                }
                if (a.out_scale != 1.0) {
                    const R sc = R(a.out_scale);
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        d[m].re *= sc;
                        d[m].im *= sc;
                    }
                }
                if constexpr (!THR) {
                    if (fh >= 0) apply_hit<R, E>(d, hf);
                }
                if constexpr (ENC) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int cls = ((T % 3) * m) % 3;
                        Ar[cls] += double(d[m].re);
                        Ai[cls] += double(d[m].im);
                    }
                }
            }
            if constexpr (ENC) {
                // sum_c w_3^c A_c, then rotate by w_3^(j mod 3)
                const double sr = Ar[0] + kW3r * (Ar[1] + Ar[2]) - kW3i * (Ai[1] - Ai[2]);
                const double si = Ai[0] + kW3r * (Ai[1] + Ai[2]) + kW3i * (Ar[1] - Ar[2]);
                const double rr = sr * rotr - si * roti, ri = sr * roti + si * rotr;
                D1r += rr;
                D1i += ri;
                if constexpr (BLK) {
                    const double w2 = double(b + 1);
                    D2r += w2 * rr;
                    D2i += w2 * ri;
                }
            }
            if constexpr (KIND == KIND_LAST) {
                // transposed store: re-map through LDS so that lanes run along
                // the C adjacent output rows of the tile
#pragma unroll
                for (int m = 0; m < E; ++m) lds[lidx(c, j + T * m)] = d[m];
                tile_sync();
                const int c2 = tid % C, j2 = tid / C;
                cx<R> *base = dst - c + c2;  // rows of one tile share the batch entry
                if constexpr (DEFER) {
#pragma unroll
                    for (int m = 0; m < E; ++m) ps[m] = lds[lidx(c2, j2 + T * m)];
                    pdst = base + (uint32_t)j2 * ostr;
                    pstr = ostr;
                    pend = L.valid;
                } else if (L.valid) {
#pragma unroll
                    for (int m = 0; m < E; ++m)
                        st_stream<R, NT_ST>(base + (uint32_t)(j2 + T * m) * ostr, lds[lidx(c2, j2 + T * m)]);
                }
                tile_sync();
            } else if constexpr (DEFER) {
#pragma unroll
                for (int m = 0; m < E; ++m) ps[m] = d[m];
                pdst = dst + (uint32_t)j * ostr;
                pstr = ostr;
                pend = L.valid;
            } else {
                if (L.valid) {
#pragma unroll
                    for (int m = 0; m < E; ++m) st_stream<R, NT_ST>(dst + (uint32_t)(j + T * m) * ostr, d[m]);
                }
            }
            if constexpr (SIGM) {
                member_check(g, b, L.valid, D1r, D1i, Ssum, 4);
                D1r = D1i = 0.0;
                Ssum = 0.0;
            }
        }  // rounds

        if constexpr (SIGR) member_check(gsig, 0, gsig < a.n_groups, D1r, D1i, Ssum, 1);
        if constexpr (BLK) {
            if constexpr (LDS_RED) {
                // partial sums through the (now idle) exchange buffer, added
                // up by one wavefront: each thread stores five values instead
                // of running five 64-bit DPP reductions
                double *part = reinterpret_cast<double *>(lds);
                tile_sync();
                part[tid] = D1r;
                part[NT + tid] = D1i;
                part[2 * NT + tid] = D2r;
                part[3 * NT + tid] = D2i;
                part[4 * NT + tid] = Ssum;
                tile_sync();
                if (tid < 64) {
                    double v[5];
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        v[q] = 0.0;
                        for (int w = tid; w < NT; w += 64) v[q] += part[q * NT + w];
                        v[q] = wave_sum_dpp(v[q], Dpp64{});
                    }
                    if (tid == 63) decide(v, g);
                }
                tile_sync();
            } else {
                double v[5] = {D1r, D1i, D2r, D2i, 0.0};
                if constexpr (NT % 64 == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = wave_sum_dpp(v[q], Dpp64{});
                    v[4] = wave_sum_dpp(Ssum, Dpp64{});
                    if ((tid & 63) == 63) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            if constexpr (RED_DEFER) redg[it & 1][tid >> 6][q] = v[q];
                            else red[tid >> 6][q] = v[q];
                        }
                    }
                } else {
                    v[4] = Ssum;
#pragma unroll
                    for (int q = 0; q < 5; ++q) v[q] = wave_sum(v[q], WIDTH);
                    if ((tid & 63) == 0) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) red[tid >> 6][q] = v[q];
                    }
                }
                if constexpr (RED_DEFER) {
                    // the previous group's sums were written before this
                    // group's exchange barriers; this group's go to the other
                    // slot, which is read only after the next group's barriers
                    if (tid == 0 && g_prev >= 0) {
                        double t[5] = {0, 0, 0, 0, 0};
                        for (int w = 0; w < WAVES; ++w)
                            for (int k = 0; k < 5; ++k) t[k] += redg[(it - 1) & 1][w][k];
                        decide(t, g_prev);
                    }
                    g_prev = g;
                    ++it;
                } else {
                    tile_sync();
                    if (tid == 0) {
                        double t[5] = {0, 0, 0, 0, 0};
                        for (int w = 0; w < WAVES; ++w)
                            for (int k = 0; k < 5; ++k) t[k] += red[w][k];
                        decide(t, g);
                    }
                    tile_sync();
                }
            }
        }
    }  // groups
    if constexpr (RED_DEFER) {
        // the last group's decision
        tile_sync();
        if (tid == 0 && g_prev >= 0) {
            double t[5] = {0, 0, 0, 0, 0};
            for (int w = 0; w < WAVES; ++w)
                for (int k = 0; k < 5; ++k) t[k] += redg[(it - 1) & 1][w][k];
            decide(t, g_prev);
        }
    }
    flush();
}

template <typename R, int M, int KIND, int FT>
__global__ void __launch_bounds__(cfg_threads(sizeof(R) == 8, M, KIND)) TFFT_PASS_OCCUPANCY
pass_kernel(PassArgs a) {
    using Cf = PassCfg<R, M, KIND, FT>;
    __shared__ PassShared<R, M, KIND, FT> sh;
    __shared__ __align__(16) cx<R> nbuf[pass_nbuf_elems<R, M, KIND, FT>()];
    // XCD-contiguous group ranges: consecutive workgroups run on different
    // XCDs, so workgroup b walks the groups of slot (b mod 8, b / 8)
    const int nwg = gridDim.x;
    int64_t wl = blockIdx.x;
    if (nwg % 8 == 0) wl = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
    const int64_t n_iter = Cf::SIGR ? (a.n_groups + Cf::C - 1) / Cf::C : a.n_groups;
    pass_body<R, M, KIND, FT, 0>(a, sh, nbuf, wl, n_iter, nwg, PassHooks{nullptr, nullptr, 0});
}

// ------------------------------------------------------- correction kernel
template <int NTH>
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    v = wave_sum(v, 64);
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) scratch[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += scratch[w];
    return t;
}

// Correction of record i (a flagged group of the pass described by `a`) by
// one workgroup of NTH threads, with C the tile width of the pass kernel that
// defined the group layout; `buf` holds M binary64 values, `scratch` NTH / 64
// doubles (LDS).  Records of another pass, task or chunk, or already acted
// on, are skipped.
template <typename R, int M, int KIND, int C, int NTH>
__device__ __forceinline__ void correct_record(const PassArgs &a, int64_t i, cx<double> *buf, double *scratch) {
    constexpr int kCorrThreads = NTH;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));  // per call (see pass_body)
    const cx<R> *in = reinterpret_cast<const cx<R> *>(a.in);
    cx<R> *out = reinterpret_cast<cx<R> *>(a.out);
    const cx<double> *cv = reinterpret_cast<const cx<double> *>(a.cvec);
    const cx<double> *w64 = reinterpret_cast<const cx<double> *>(a.stw64);
    {
        const DevRecord rec = a.recs[i];
        // records of this pass and of this launch's groups (a chunk of the
        // batch covers groups g_base .. g_base + n_groups - 1)
        if (rec.pass != a.pass || rec.task != a.task || rec.action != 1) return;
        if (rec.group < a.g_base || rec.group >= a.g_base + a.n_groups) return;
        const int64_t g = rec.group - a.g_base;

        // applied output twiddle of member loc at output k (1 outside strided passes)
        auto applied = [&](const MemberLoc &L, int k) -> cx<double> {
            if constexpr (KIND == KIND_STRIDED) {
                cx<double> w = itw(a, (int64_t(k) * L.tw_i * a.tw_scale) & (a.n - 1));
                if (a.conj_out) w.im = -w.im;
                return w;
            } else {
                return cx<double>{1.0, 0.0};
            }
        };
        auto load_in = [&](const MemberLoc &L, int n) -> cx<double> {
            const cx<R> x = ldg(in + L.in_off + (uint32_t)n * L.in_stride);
            return {double(x.re), double(x.im)};
        };
        auto load_out = [&](const MemberLoc &L, int k) -> cx<double> {
            const cx<R> y = ldg(out + L.out_off + (uint32_t)k * L.out_stride);
            return {double(y.re), double(y.im)};
        };
        auto ek = [](int k) -> cx<double> {
            const int r = k % 3;
            return {r == 0 ? 1.0 : kW3r, r == 0 ? 0.0 : (r == 1 ? kW3i : -kW3i)};
        };

        // location: quotient of the residuals, else per-signal residuals
        int jl = rec.member;
        if (jl >= a.G || (jl >= 0 && !member_loc<M, KIND, C>(a, g, jl).valid)) jl = -1;
        int method = rec.method == 4 ? 4 : (jl >= 0 ? 1 : 0);
        // a one-sided record (a sub-signal checked alone) is recomputed from
        // its own input: the sums below then take that member only
        const int only = rec.method == 4 ? jl : -1;
        if (jl < 0) {
            int ncand = 0, cand = -1;
            for (int b = 0; b < a.G; ++b) {
                const MemberLoc L = member_loc<M, KIND, C>(a, g, b);
                if (!L.valid) continue;
                double dr = 0.0, di = 0.0, sb = 0.0;
                for (int n = tid; n < M; n += kCorrThreads) {
                    const cx<double> x = load_in(L, n);
                    const cx<double> cn = cv[n];
                    dr -= cn.re * x.re - cn.im * x.im;
                    di -= cn.re * x.im + cn.im * x.re;
                    sb += x.re * x.re + x.im * x.im;
                    const cx<double> y = cmulconj(load_out(L, n), applied(L, n));
                    const cx<double> e = ek(n);
                    dr += e.re * y.re - e.im * y.im;
                    di += e.re * y.im + e.im * y.re;
                }
                dr = block_sum<NTH>(dr, scratch);
                di = block_sum<NTH>(di, scratch);
                sb = block_sum<NTH>(sb, scratch);
                const double taub = a.tau_coef * sqrt(sb);
                if (!(sqrt(dr * dr + di * di) <= taub)) {
                    ++ncand;
                    cand = b;
                }
            }
            if (ncand == 1) {
                jl = cand;
                method = 2;
            }
        }

        // Member sums are taken with lanes along the C adjacent members of a
        // tile when those are adjacent in memory (strided passes; outputs of
        // the last pass), else along the positions; the C lanes that share a
        // position are then summed with lane shuffles.
        constexpr int CL = (KIND == KIND_ROWS) ? 1 : C;
        constexpr bool IN_ALONG_MEMBERS = KIND == KIND_STRIDED;
        constexpr bool OUT_ALONG_MEMBERS = KIND != KIND_ROWS;
        // Members are visited in batches of CU whose loads are all issued
        // before any is summed (a missing member reads member 0, a valid
        // location, and contributes zero), so the group's rows stream in
        // rather than arriving one latency at a time.
        constexpr int CU = TFFT_CORRECT_BATCH;
        const MemberLoc L0 = member_loc<M, KIND, C>(a, g, 0);
        auto member_sum = [&](bool along_members, int n, auto &&value) -> cx<double> {
            // sum over the members of `value(L, n)`; the calling lanes share n
            // in groups of CL adjacent lanes when along_members
            const int first = along_members ? tid % CL : 0;
            const int stride = along_members ? CL : 1;
            cx<double> acc{0.0, 0.0};
            for (int b0 = first; b0 < a.G; b0 += CU * stride) {
                cx<double> v[CU];
#pragma unroll
                for (int u = 0; u < CU; ++u) {
                    const int bm = b0 + u * stride;
                    const MemberLoc Lb = member_loc<M, KIND, C>(a, g, bm < a.G ? bm : 0);
                    const bool ok = bm < a.G && Lb.valid && (only < 0 || bm == only);
                    v[u] = value(ok ? Lb : L0, bm, n);
                    if (!ok) v[u] = cx<double>{0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < CU; ++u) acc = cadd(acc, v[u]);
            }
            if (along_members) {
                for (int off = 1; off < CL; off *= 2) {
                    acc.re += __shfl_xor(acc.re, off, 64);
                    acc.im += __shfl_xor(acc.im, off, 64);
                }
            }
            return acc;
        };

        // transform of the combined input, fp64: radix-2 decimation in time in
        // place in LDS (inputs stored at bit-reversed positions)
        constexpr int LOGM = ilog2c(M);
        {
            const int step = IN_ALONG_MEMBERS ? kCorrThreads / CL : kCorrThreads;
            const int n0 = IN_ALONG_MEMBERS ? tid / CL : tid;
            for (int n = n0; n < M; n += step) {
                cx<double> acc = member_sum(IN_ALONG_MEMBERS, n, [&](const MemberLoc &L, int, int nn) {
                    return load_in(L, nn);
                });
                if (a.conj_in) acc.im = -acc.im;
                const int rn = LOGM == 0 ? 0 : (int)(__brev((unsigned)n) >> (32 - LOGM));
                if (!IN_ALONG_MEMBERS || tid % CL == 0) buf[rn] = acc;
            }
        }
        __syncthreads();
        for (int half = 1; half < M; half *= 2) {
            for (int t = tid; t < M / 2; t += kCorrThreads) {
                const int kk = t & (half - 1);
                const int i0 = (t - kk) * 2 + kk, i1 = i0 + half;
                const cx<double> w = w64[kk * (M / (2 * half))];
                const cx<double> x0 = buf[i0];
                const cx<double> x1 = cmul(buf[i1], w);
                buf[i0] = cadd(x0, x1);
                buf[i1] = csub(x0, x1);
            }
            __syncthreads();
        }
        for (int kk = tid; kk < M; kk += kCorrThreads) {
            cx<double> p = buf[kk];
            if (a.conj_out) p.im = -p.im;
            p.re *= a.out_scale;
            p.im *= a.out_scale;
            buf[kk] = p;
        }
        __syncthreads();

        // P - sum of the (un-twiddled) outputs of the members other than jl
        // (jl < 0: of all members), in place
        {
            const int step = OUT_ALONG_MEMBERS ? kCorrThreads / CL : kCorrThreads;
            const int k0 = OUT_ALONG_MEMBERS ? tid / CL : tid;
            for (int kk = k0; kk < M; kk += step) {
                const cx<double> s = member_sum(OUT_ALONG_MEMBERS, kk, [&](const MemberLoc &L, int bm, int k2) {
                    const cx<double> y = cmulconj(load_out(L, k2), applied(L, k2));
                    return bm == jl ? cx<double>{0.0, 0.0} : y;
                });
                if (!OUT_ALONG_MEMBERS || tid % CL == 0) buf[kk] = csub(buf[kk], s);
            }
        }
        __syncthreads();

        int action;
        if (jl >= 0) {
            const MemberLoc Lj = member_loc<M, KIND, C>(a, g, jl);
            for (int kk = tid; kk < M; kk += kCorrThreads) {
                const cx<double> y = cmul(buf[kk], applied(Lj, kk));
                stg(out + Lj.out_off + (uint32_t)kk * Lj.out_stride, cx<R>{R(y.re), R(y.im)});
            }
            action = 2;
        } else {
            double nrm = 0.0;
            for (int kk = tid; kk < M; kk += kCorrThreads) {
                const cx<double> v = buf[kk];
                nrm += v.re * v.re + v.im * v.im;
            }
            nrm = block_sum<NTH>(nrm, scratch);
            action = (sqrt(nrm) <= rec.tau) ? 3 : 4;
        }
        if (tid == 0) {
            a.recs[i].member = jl;
            a.recs[i].method = method;
            a.recs[i].action = action;
            atomicAdd(action == 2 ? &a.rep->corrected : action == 3 ? &a.rep->benign : &a.rep->uncorrectable, 1ULL);
        }
        __syncthreads();
    }
}

constexpr int kCorrThreads = 256;

template <typename R, int M, int KIND>
__global__ void __launch_bounds__(kCorrThreads) correct_kernel(PassArgs a) {
    constexpr int C = cfg_C(sizeof(R) == 8, M, KIND);
    __shared__ cx<double> buf[M];  // the binary64 transform, in place
    __shared__ double scratch[kCorrThreads / 64];
    unsigned long long nrec = a.rep->n_flag;
    if ((int64_t)nrec > a.rec_cap) nrec = a.rec_cap;
    for (int64_t i = blockIdx.x; i < (int64_t)nrec; i += gridDim.x)
        correct_record<R, M, KIND, C, kCorrThreads>(a, i, buf, scratch);
}

// ------------------------------------------------------------- dispatch
template <typename R, int M, int KIND, int FT>
static hipError_t launch_one(const PassArgs &a, int grid, hipStream_t st) {
    constexpr int NT = cfg_threads(sizeof(R) == 8, M, KIND);
    hipLaunchKernelGGL((pass_kernel<R, M, KIND, FT>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename R, int M, int KIND>
static hipError_t launch_kind(int ft, const PassArgs &a, int grid, hipStream_t st) {
    if (ft == FT_BLOCK) return launch_one<R, M, KIND, FT_BLOCK>(a, grid, st);
    if (ft == FT_NONE) return launch_one<R, M, KIND, FT_NONE>(a, grid, st);
    if (ft == FT_THREAD) {
        // butterfly encodings exist for radix 2, 4 and 8 (plans of the
        // thread-level scheme use no larger thread radix)
        if constexpr (cfg_E(sizeof(R) == 8, M, KIND) <= 8) return launch_one<R, M, KIND, FT_THREAD>(a, grid, st);
        else return hipErrorInvalidValue;
    }
    if (ft == FT_SIGNAL) return launch_one<R, M, KIND, FT_SIGNAL>(a, grid, st);
    return hipErrorInvalidValue;
}

template <typename R, int M>
hipError_t launch_m(int kind, int ft, const PassArgs &a, int grid, hipStream_t st) {
    if (kind == KIND_ROWS) return launch_kind<R, M, KIND_ROWS>(ft, a, grid, st);
    if constexpr (M >= 16 && M <= 1024) {
        if (kind == KIND_STRIDED) return launch_kind<R, M, KIND_STRIDED>(ft, a, grid, st);
        if (kind == KIND_LAST) return launch_kind<R, M, KIND_LAST>(ft, a, grid, st);
    }
    return hipErrorInvalidValue;
}

template <typename R, int M>
hipError_t correct_m(int kind, const PassArgs &a, int grid, hipStream_t st) {
    if (kind == KIND_ROWS) {
        hipLaunchKernelGGL((correct_kernel<R, M, KIND_ROWS>), dim3(grid), dim3(kCorrThreads), 0, st, a);
        return hipGetLastError();
    }
    if constexpr (M >= 16 && M <= 1024) {
        if (kind == KIND_STRIDED) {
            hipLaunchKernelGGL((correct_kernel<R, M, KIND_STRIDED>), dim3(grid), dim3(kCorrThreads), 0, st, a);
            return hipGetLastError();
        }
        if (kind == KIND_LAST) {
            hipLaunchKernelGGL((correct_kernel<R, M, KIND_LAST>), dim3(grid), dim3(kCorrThreads), 0, st, a);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

template <typename R, int M, int KIND, int FT>
static int occ_one() {
    int n = 0;
    constexpr int NT = cfg_threads(sizeof(R) == 8, M, KIND);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pass_kernel<R, M, KIND, FT>, NT, 0) != hipSuccess) return 0;
    return n;
}

template <typename R, int M>
int occ_m(int kind, int ft) {
    if (kind == KIND_ROWS) return ft ? occ_one<R, M, KIND_ROWS, FT_BLOCK>() : occ_one<R, M, KIND_ROWS, FT_NONE>();
    if constexpr (M >= 16 && M <= 1024) {
        if (kind == KIND_STRIDED)
            return ft ? occ_one<R, M, KIND_STRIDED, FT_BLOCK>() : occ_one<R, M, KIND_STRIDED, FT_NONE>();
        if (kind == KIND_LAST) return ft ? occ_one<R, M, KIND_LAST, FT_BLOCK>() : occ_one<R, M, KIND_LAST, FT_NONE>();
    }
    return 0;
}

// Explicit instantiation (one translation unit per pair) and the matching
// declarations that keep the dispatching unit from instantiating them.
#define TFFT_INSTANTIATE_M(R, M)                                                         \
    template hipError_t launch_m<R, M>(int, int, const PassArgs &, int, hipStream_t); \
    template hipError_t correct_m<R, M>(int, const PassArgs &, int, hipStream_t);     \
    template int occ_m<R, M>(int, int);
#define TFFT_EXTERN_M(R, M)                                                                     \
    extern template hipError_t launch_m<R, M>(int, int, const PassArgs &, int, hipStream_t); \
    extern template hipError_t correct_m<R, M>(int, const PassArgs &, int, hipStream_t);     \
    extern template int occ_m<R, M>(int, int);
#define TFFT_FOR_EACH_M(X, R) X(R, 2) X(R, 4) X(R, 8) X(R, 16) X(R, 32) X(R, 64) X(R, 128) X(R, 256) \
    X(R, 512) X(R, 1024) X(R, 2048) X(R, 4096) X(R, 8192)

}  // namespace tfft
