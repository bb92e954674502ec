// Host side of the fault-tolerant batched FFT: plans, tables, the C ABI.
//
// Every twiddle and checksum vector is generated here in binary64 from exact
// integer angle arguments and rounded once to the element type
// (TurboFFT Section IV-A.3 keeps twiddles in global memory because computing
// them in the kernel costs time; here they are tables for both precisions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "../../include/tfft.h"
#include "tfft_internal.h"

using namespace tfft;
using cd = std::complex<double>;


static_assert(kScratchBytes == TFFT_SCRATCH_BYTES, "static scratch size as declared in the header");

namespace {

// exp(-2 pi i t / n) for integers t, n.  The argument is split into a
// quadrant q and a remainder r (4 t = q n + r, 0 <= r < n, exact integer
// arithmetic) so libm only sees angles in [0, pi/4]; the quadrant is applied
// as an exact multiplication by (-i)^q.
cd unit_root(int64_t t, int64_t n) {
    t %= n;
    if (t < 0) t += n;
    const __int128 four_t = (__int128)4 * t;
    const int q = (int)(four_t / n);
    const int64_t r = (int64_t)(four_t - (__int128)q * n);  // angle within quadrant = (pi/2) r / n
    double c, s;
    if (2 * r <= n) {
        const double ang = (M_PI / 2.0) * ((double)r / (double)n);
        c = std::cos(ang);
        s = std::sin(ang);
    } else {
        const double ang = (M_PI / 2.0) * ((double)(n - r) / (double)n);
        c = std::sin(ang);
        s = std::cos(ang);
    }
    if (r == 0) {
        c = 1.0;
        s = 0.0;
    }
    // exp(-i (q pi/2 + phi)) = (-i)^q (c - i s)
    cd w(c, -s);
    switch (q & 3) {
        case 1: w = cd(w.imag(), -w.real()); break;    // * (-i)
        case 2: w = cd(-w.real(), -w.imag()); break;   // * (-1)
        case 3: w = cd(-w.imag(), w.real()); break;    // * (+i)
        default: break;
    }
    return w;
}

struct PassPlan {
    int M = 0, kind = 0, E = 0, C = 0, G = 0, rb = 1, stages = 0;
    int64_t n_strips = 1, n_groups = 0, n_outer = 0;
    int64_t L = 0, rows = 0, tw_scale = 1;
    int S = 1, O = 1, m1 = 1, m2 = 1;
    int grid = 0;
    void *d_stw = nullptr;       // element-type stage twiddles
    double *d_stw64 = nullptr;   // fp64 stage twiddles
    double *d_cfwd = nullptr;    // checksum vector, forward
    double *d_cinv = nullptr;    // checksum vector, inverse (scaled for the last pass)
    double *d_cinv_unscaled = nullptr;
    int32_t *d_fault_head = nullptr;
    DevFault *d_faults = nullptr;
    double tau_coef = 0.0;
};

}  // namespace

struct tfft_plan_s {
    int device = 0;
    int64_t n = 0, batch = 0;
    int dtype = 0;
    uint32_t flags = 0;
    double kappa = 16.0;
    int scheme = TFFT_SCHEME_BLOCK;
    int passes = 0;
    int lens[kMaxPasses] = {0, 0, 0};
    PassPlan pass[kMaxPasses];
    double *d_itw_lo = nullptr, *d_itw_hi = nullptr;
    int itw_bits = 0;
    void *d_work = nullptr;
    size_t work_bytes = 0;
    DevReport *d_rep = nullptr;
    DevRecord *d_recs = nullptr;
    int64_t rec_cap = 0;
    DevReport *rep_last = nullptr;  // report buffers of the last execution (the plan's or the static scratch)
    DevRecord *recs_last = nullptr;
    hipStream_t last_stream = nullptr;
    int executed = 0;
    int last_mode = 0;
    int64_t nfaults = 0;
    int64_t *d_sig_off = nullptr;  // ragged class: element offset of each signal (device)
    int64_t extent = 0;            // elements spanned by the input / output buffers
    int timing = 0;              // record events around each launch
    int timed_last = 0;          // the last execution was timed
    hipEvent_t ev[2 * kMaxPasses + 1] = {};
    int launched_correct = 0;
    int64_t chunk = 0;           // multi-pass plans: signals per chunk of the batch (= batch: no chunking)
    int persistent = 0;          // shaped for the persistent ragged kernel (tiles of 512 threads)
};

namespace {

int ilog2_64(int64_t x) {
    int k = 0;
    while ((int64_t(1) << k) < x) ++k;
    return k;
}

template <typename T>
int upload(T **dst, const std::vector<T> &v) {
    if (hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(1, v.size())) != hipSuccess) {
        *dst = nullptr;
        return TFFT_E_NOMEM;
    }
    if (!v.empty() && hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return TFFT_E_HIP;
    return TFFT_OK;
}

#ifndef TFFT_GROUP_SMALL
#define TFFT_GROUP_SMALL 64
#endif
// One-pass group size: the common path favours large groups (fewer
// reductions), a correction re-reads the whole group (cost proportional to G).
int default_group(int M) {
    if (M >= 4096) return 16;
    if (M >= 2048) return 32;
    return TFFT_GROUP_SMALL;
}

// c_n = s sum_k w_3^k w_M^{+-k n}.  Each term is w_{3M}^{k q} with
// q = (M +- 3n) mod 3M, so the sum is geometric: (1 - w_3^M) / (1 - w_{3M}^q).
// Writing w_{3M}^q = v^2 with v = w_{6M}^q, 1 - v^2 = v (conj(v) - v) =
// -2i Im(v) v, which has no cancellation; v comes from the exactly reduced
// root, so each entry is within a few ulp.
std::vector<double> checksum_vec(int M, bool inverse, double scale) {
    std::vector<double> out(2 * (size_t)M);
    const cd num = 1.0 - unit_root(M % 3, 3);
    const int64_t M3 = 3 * (int64_t)M;
    for (int n = 0; n < M; ++n) {
        int64_t q = ((int64_t)M + (inverse ? -3 : 3) * (int64_t)n) % M3;
        if (q < 0) q += M3;
        const cd v = unit_root(q, 2 * M3);
        const cd c = scale * num * std::conj(v) * cd(0.0, 1.0 / (2.0 * v.imag()));
        out[2 * n] = c.real();
        out[2 * n + 1] = c.imag();
    }
    return out;
}

// Geometry of pass idx (no device call): thread radix, tile, checksum
// groups, workgroups and the threshold coefficient.
int shape_pass(tfft_plan_s *p, int idx, int M, int kind, int Guser, int grid_scale) {
    PassPlan &P = p->pass[idx];
    const int fp64 = p->dtype == TFFT_C128;
    P.M = M;
    P.kind = kind;
    P.E = cfg_E(fp64, M, kind);
    // the persistent kernel widens every tile to 512 threads (PassCfg with NTHR = 512)
    P.C = p->persistent ? std::max(1, kPersistThreads / (M / P.E)) : cfg_C(fp64, M, kind);
    P.stages = n_stages(M, P.E);
    const int G0 = Guser > 0 ? Guser : (kind == KIND_ROWS ? default_group(M) : 64);
    int64_t tiles;  // workgroup iterations of the pass
    if (kind == KIND_ROWS && p->scheme == TFFT_SCHEME_SIGNAL) {
        // one-sided: every signal is a group of its own; tiles of C signals
        P.G = 1;
        P.rb = 1;
        P.n_strips = 1;
        P.n_outer = p->batch;
        P.n_groups = p->batch;
        tiles = (p->batch + P.C - 1) / P.C;
    } else if (kind == KIND_ROWS) {
        if (G0 % P.C != 0) return TFFT_E_UNSUPPORTED;
        P.G = G0;
        P.rb = 1;
        P.n_strips = 1;
        P.n_outer = p->batch;
        P.n_groups = (p->batch + P.G - 1) / P.G;
        tiles = P.n_groups;
    } else {
        int64_t n_sub;  // sub-signals per outer unit
        if (kind == KIND_STRIDED) {
            P.L = 1;
            for (int q = idx; q < p->passes; ++q) P.L *= p->lens[q];
            P.S = (int)(P.L / M);
            P.O = (int)(p->n / P.L);
            P.tw_scale = p->n / P.L;
            P.n_outer = p->batch * P.O;
            n_sub = P.S;
        } else {
            P.rows = p->n / M;
            P.m1 = p->lens[0];
            P.m2 = p->passes == 3 ? p->lens[1] : 1;
            P.n_outer = p->batch;
            n_sub = P.rows;
        }
        if (n_sub % P.C != 0) return TFFT_E_UNSUPPORTED;
        P.rb = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(1, G0 / P.C), P.n_outer));
        P.G = P.C * P.rb;
        P.n_strips = n_sub / P.C;
        P.n_groups = P.n_strips * ((P.n_outer + P.rb - 1) / P.rb);
        tiles = P.n_groups;
    }
    int64_t cap = std::max<int64_t>(8, (int64_t)TFFT_GRID_THREADS / cfg_threads(fp64, M, kind));
    if (TFFT_GRID_MP_BIG_M > 0 && kind != KIND_ROWS && M >= TFFT_GRID_MP_BIG_M) cap *= 2;
    if (TFFT_GRID_MULT > 0) {
        // a persistent launch: TFFT_GRID_MULT x the workgroups resident at once
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
        const int occ = std::max(1, pass_occupancy(fp64, M, kind, 1));
        cap = std::max<int64_t>(8, (int64_t)TFFT_GRID_MULT * occ * std::max(1, cus));
    }
    if (grid_scale > 0) cap <<= grid_scale;
    if (grid_scale < 0) cap = std::max<int64_t>(8, cap >> (-grid_scale));
    int64_t grid = std::min<int64_t>(tiles, cap);
    if (grid >= 8) grid = (grid + 7) / 8 * 8;
    P.grid = (int)std::max<int64_t>(1, grid);
    const double u = fp64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    P.tau_coef = p->kappa * u * std::sqrt(std::max(1.0, (double)ilog2_64(M))) * std::sqrt((double)M);
    return TFFT_OK;
}

// Tables of pass idx (stage twiddles in the element type and in fp64, the
// checksum vectors of both directions), generated in fp64 and uploaded.
int upload_pass(tfft_plan_s *p, int idx) {
    PassPlan &P = p->pass[idx];
    const int fp64 = p->dtype == TFFT_C128;
    const int M = P.M;
    // stage twiddles w_M^t, t < M
    std::vector<double> w64(2 * (size_t)M);
    for (int t = 0; t < M; ++t) {
        const cd w = unit_root(t, M);
        w64[2 * t] = w.real();
        w64[2 * t + 1] = w.imag();
    }
    int rc;
    if (fp64) {
        if ((rc = upload((double **)&P.d_stw, w64)) != TFFT_OK) return rc;
    } else {
        std::vector<float> w32(w64.begin(), w64.end());
        if ((rc = upload((float **)&P.d_stw, w32)) != TFFT_OK) return rc;
    }
    if ((rc = upload(&P.d_stw64, w64)) != TFFT_OK) return rc;
    const bool last = idx == p->passes - 1;
    if ((rc = upload(&P.d_cfwd, checksum_vec(M, false, 1.0))) != TFFT_OK) return rc;
    if ((rc = upload(&P.d_cinv_unscaled, checksum_vec(M, true, 1.0))) != TFFT_OK) return rc;
    if ((rc = upload(&P.d_cinv, checksum_vec(M, true, last ? 1.0 / (double)p->n : 1.0))) != TFFT_OK) return rc;
    return TFFT_OK;
}

void free_plan(tfft_plan_s *p) {
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    for (auto &P : p->pass) {
        (void)hipFree(P.d_stw);
        (void)hipFree(P.d_stw64);
        (void)hipFree(P.d_cfwd);
        (void)hipFree(P.d_cinv);
        (void)hipFree(P.d_cinv_unscaled);
        (void)hipFree(P.d_fault_head);
        (void)hipFree(P.d_faults);
    }
    (void)hipFree(p->d_itw_lo);
    (void)hipFree(p->d_itw_hi);
    (void)hipFree(p->d_work);
    (void)hipFree(p->d_rep);
    (void)hipFree(p->d_recs);
    (void)hipFree(p->d_sig_off);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    delete p;
}

int clear_faults(tfft_plan_s *p) {
    for (auto &P : p->pass) {
        (void)hipFree(P.d_fault_head);
        (void)hipFree(P.d_faults);
        P.d_fault_head = nullptr;
        P.d_faults = nullptr;
    }
    p->nfaults = 0;
    return TFFT_OK;
}

struct Guard {
    int prev = 0;
    explicit Guard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Guard() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != prev) (void)hipSetDevice(prev);
    }
};

// Geometry of pass P restricted to signals [c0, c0 + nb) of the batch: the
// launch's outer units, groups, first group and workgroups.  Chunks start at
// multiples of 64 signals, so no checksum group straddles two chunks.
struct ChunkGeom {
    int64_t n_outer, n_groups, g_base;
    int grid;
};

ChunkGeom chunk_geom(const tfft_plan_s *p, const PassPlan &P, int64_t c0, int64_t nb) {
    ChunkGeom c;
    int64_t tiles;
    if (P.kind == KIND_ROWS) {
        c.n_outer = nb;
        if (P.G == 1 && p->scheme == TFFT_SCHEME_SIGNAL) {
            c.n_groups = nb;
            c.g_base = c0;
            tiles = (nb + P.C - 1) / P.C;
        } else {
            c.n_groups = (nb + P.G - 1) / P.G;
            c.g_base = c0 / P.G;
            tiles = c.n_groups;
        }
    } else {
        const int64_t per = P.kind == KIND_STRIDED ? P.O : 1;  // outer units per signal
        c.n_outer = nb * per;
        c.n_groups = P.n_strips * ((c.n_outer + P.rb - 1) / P.rb);
        c.g_base = P.n_strips * (c0 * per / P.rb);
        tiles = c.n_groups;
    }
    int64_t grid = std::min<int64_t>(tiles, P.grid);
    if (grid >= 8) grid = (grid + 7) / 8 * 8;
    c.grid = (int)std::max<int64_t>(1, grid);
    return c;
}

// Arguments of the launch of pass i over the signals described by cg (nb
// signals from cin / cout, the caller's buffers from the chunk's first
// signal, or the ragged offset table sig), with the plan's tables and the
// given report buffers.
PassArgs pass_args(const tfft_plan_s *p, int i, const ChunkGeom &cg, int64_t nb, const void *cin, void *cout,
                   void *work, const int64_t *sig, bool inverse, int mode, DevReport *rep, DevRecord *recs) {
    PassArgs A;
    std::memset(&A, 0, sizeof(A));
    const PassPlan &P = p->pass[i];
    const bool last = i == p->passes - 1;
    const int fp64 = p->dtype == TFFT_C128;
    // every pass reads a buffer it does not write, so a flagged group can
    // re-read its inputs: 1 pass in->out; 2 passes in->work->out;
    // 3 passes in->out->work->out (out holds the pass-1 result meanwhile)
    if (p->passes == 1) {
        A.in = cin;
        A.out = cout;
    } else if (p->passes == 2) {
        A.in = i == 0 ? cin : work;
        A.out = i == 0 ? work : cout;
    } else {
        A.in = i == 0 ? cin : (i == 1 ? (const void *)cout : work);
        A.out = i == 1 ? work : cout;
    }
    A.batch = nb;
    A.n = p->n;
    A.L = P.L;
    A.S = P.S;
    A.O = P.O;
    A.rows = P.rows;
    A.m1 = P.m1;
    A.m2 = P.m2;
    A.tw_scale = P.tw_scale;
    A.n_outer = cg.n_outer;
    // ragged classes address their signals through the offset table in
    // the user buffers; the workspace is always dense [chunk][n]
    A.in_sig = (A.in == cin || A.in == (const void *)cout) ? sig : nullptr;
    A.out_sig = (A.out == cout) ? sig : nullptr;
    A.G = P.G;
    A.rb = P.rb;
    A.n_strips = P.n_strips;
    A.m1_log2 = ilog2_64(P.m1);
    A.ns_log2 = ilog2_64(P.n_strips);
    A.o_log2 = ilog2_64(P.O);
    A.n_groups = cg.n_groups;
    A.g_base = cg.g_base;
    A.conj_in = inverse ? 1 : 0;
    A.conj_out = inverse ? 1 : 0;
    A.out_scale = (inverse && last && !(p->flags & TFFT_INVERSE_UNSCALED)) ? 1.0 / (double)p->n : 1.0;
    A.cvec = !inverse ? P.d_cfwd : ((p->flags & TFFT_INVERSE_UNSCALED) ? P.d_cinv_unscaled : P.d_cinv);
    A.stw = P.d_stw;
    A.stw64 = P.d_stw64;
    A.itw_lo = p->d_itw_lo;
    A.itw_hi = p->d_itw_hi;
    A.itw_bits = p->itw_bits;
    A.pass = i;
    A.tau_coef = P.tau_coef * A.out_scale;  // the outputs' rounding noise scales with them
    A.rep = rep;
    A.recs = recs;
    A.rec_cap = p->rec_cap;
    A.fault_head = P.d_fault_head;
    A.faults = P.d_faults;
    A.kappa_u = p->kappa * (fp64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
    A.fix = mode == TFFT_FT_CORRECT;
    return A;
}

// Device buffers of one execution: the report counters, the records and the
// multi-pass workspace (the plan's own, or parts of the static scratch).
struct ExecBufs {
    DevReport *rep;
    DevRecord *recs;
    void *work;
};

int exec(tfft_plan_s *p, const void *d_in, void *d_out, int mode, void *stream, bool inverse,
         const ExecBufs *bufs = nullptr) {
    if (!p || !d_in || !d_out) return TFFT_E_INVALID;
    if (mode < TFFT_FT_OFF || mode > TFFT_FT_CORRECT) return TFFT_E_INVALID;
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 15)) return TFFT_E_INVALID;
    const size_t esz = p->dtype == TFFT_C128 ? 16 : 8;
    const size_t bytes = (size_t)p->extent * esz;
    const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
    // in place (d_in == d_out) works pass by pass: a tile is read before the
    // same workgroup writes it.  A correction re-reads the inputs of its pass,
    // which in place survive only in two-pass plans (in -> workspace -> out);
    // the thread-level scheme corrects in registers.
    if (a == b) {
        if (mode == TFFT_FT_CORRECT && p->passes != 2 && p->scheme != TFFT_SCHEME_THREAD) return TFFT_E_UNSUPPORTED;
    } else if ((a < b ? b - a : a - b) < bytes) {
        return TFFT_E_INVALID;  // partial overlap
    }
    void *work = bufs ? bufs->work : p->d_work;
    DevReport *rep = bufs ? bufs->rep : p->d_rep;
    DevRecord *recs = bufs ? bufs->recs : p->d_recs;
    if (p->passes > 1 && !work) return TFFT_E_STATE;
    Guard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    const int fp64 = p->dtype == TFFT_C128;
    const int ft = mode != TFFT_FT_OFF;
    if (launch_reset(rep, st) != hipSuccess) return TFFT_E_HIP;
    // one chunk (the whole batch) unless the plan chunks its multi-pass batch
    const int64_t chunk = (p->passes > 1 && p->chunk > 0) ? p->chunk : p->batch;
    const bool timed = p->timing != 0;
    const bool per_pass_events = timed && chunk >= p->batch;
    if (timed && hipEventRecord(p->ev[0], st) != hipSuccess) return TFFT_E_HIP;
    const int scheme_ft = !ft ? FT_NONE
                              : (p->scheme == TFFT_SCHEME_SIGNAL ? FT_SIGNAL
                                                                 : (p->scheme == TFFT_SCHEME_THREAD ? FT_THREAD : FT_BLOCK));
    const bool correct = mode == TFFT_FT_CORRECT && p->scheme != TFFT_SCHEME_THREAD;
    for (int64_t c0 = 0; c0 < p->batch; c0 += chunk) {
        const int64_t nb = std::min(chunk, p->batch - c0);
        // the caller's buffers from signal c0 on (dense: an offset pointer;
        // ragged class: the offset table from entry c0 on)
        const size_t off = p->d_sig_off ? 0 : (size_t)c0 * (size_t)p->n * esz;
        const void *cin = (const char *)d_in + off;
        void *cout = (char *)d_out + off;
        const int64_t *sig = p->d_sig_off ? p->d_sig_off + c0 : nullptr;
        for (int i = 0; i < p->passes; ++i) {
            const PassPlan &P = p->pass[i];
            const ChunkGeom cg = chunk_geom(p, P, c0, nb);
            const PassArgs A = pass_args(p, i, cg, nb, cin, cout, work, sig, inverse, mode, rep, recs);
            if (launch_pass(fp64, P.M, P.kind, scheme_ft, A, cg.grid, st) != hipSuccess) return TFFT_E_HIP;
            if (per_pass_events && hipEventRecord(p->ev[1 + 2 * i], st) != hipSuccess) return TFFT_E_HIP;
            if (correct) {
                // one workgroup per possible record, at most TFFT_CORRECT_GRID; a workgroup
                // with no record of this pass and chunk exits at once
                const int cgrid = (int)std::min<int64_t>(TFFT_CORRECT_GRID, std::max<int64_t>(1, cg.n_groups));
                if (launch_correct(fp64, P.M, P.kind, A, cgrid, st) != hipSuccess) return TFFT_E_HIP;
            }
            if (per_pass_events && hipEventRecord(p->ev[2 + 2 * i], st) != hipSuccess) return TFFT_E_HIP;
        }
    }
    if (timed && !per_pass_events && hipEventRecord(p->ev[2 * p->passes], st) != hipSuccess) return TFFT_E_HIP;
    p->timed_last = timed ? (per_pass_events ? 1 : 2) : 0;
    p->launched_correct = correct;
    p->rep_last = rep;
    p->recs_last = recs;
    p->last_stream = st;
    p->executed = 1;
    p->last_mode = mode;
    return TFFT_OK;
}

}  // namespace

extern "C" {

int tfft_version(void) { return TFFT_VERSION; }

int tfft_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream) {
    if (!d_dst || !d_src || (((uintptr_t)d_dst | (uintptr_t)d_src) & 15)) return TFFT_E_INVALID;
    const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
    if ((a < b ? b - a : a - b) < bytes) return TFFT_E_INVALID;  // overlapping
    if (bytes == 0) return TFFT_OK;
    return launch_stream_copy(d_dst, d_src, bytes, (hipStream_t)hip_stream) == hipSuccess ? TFFT_OK : TFFT_E_HIP;
}

const char *tfft_status_string(int s) {
    switch (s) {
        case TFFT_OK: return "ok";
        case TFFT_UNCORRECTABLE: return "completed; a flagged group could not be corrected";
        case TFFT_E_INVALID: return "invalid argument";
        case TFFT_E_UNSUPPORTED: return "unsupported configuration";
        case TFFT_E_NOMEM: return "out of memory";
        case TFFT_E_HIP: return "HIP runtime error";
        case TFFT_E_STATE: return "call out of order";
        case TFFT_E_SCRATCH: return "the execution needs more than the library's static scratch (64 MiB per device)";
        default: return "unknown status";
    }
}

}  // extern "C"

namespace {

// Validation and geometry of a plan (no device call): *p is filled with the
// pass decomposition and every pass's shape.
int shape_plan(tfft_plan_s *p, int64_t n, int64_t batch, int dtype, const tfft_options *opt, bool ragged) {
    if (n < 2 || n > (int64_t(1) << 24) || (n & (n - 1)) != 0) return TFFT_E_INVALID;
    if (batch < 1 || dtype < TFFT_C64 || dtype > TFFT_C128) return TFFT_E_INVALID;
    const size_t esz = dtype == TFFT_C128 ? 16 : 8;
    if ((uint64_t)batch > (UINT64_MAX / 4) / ((uint64_t)n * esz)) return TFFT_E_INVALID;
    const uint32_t flags = opt ? opt->flags : 0;
    const int Guser = opt ? opt->group : 0;
    if (Guser < 0 || Guser > 64 || (Guser & (Guser - 1)) != 0) return TFFT_E_INVALID;
    if (opt && (opt->kappa < 0 || !std::isfinite(opt->kappa))) return TFFT_E_INVALID;
    if (flags & ~(uint32_t)(TFFT_INVERSE_UNSCALED | TFFT_PERSISTENT | TFFT_PERSIST_INTERLEAVE | TFFT_PERSIST_ONE_QUEUE))
        return TFFT_E_INVALID;
    if ((flags & TFFT_PERSISTENT) && !ragged) return TFFT_E_INVALID;  // a ragged-batch mode
    if ((flags & (TFFT_PERSIST_INTERLEAVE | TFFT_PERSIST_ONE_QUEUE)) && !(flags & TFFT_PERSISTENT))
        return TFFT_E_INVALID;
    const int split = opt ? opt->split : 0;
    if (split < 0 || split > 1) return TFFT_E_INVALID;
    const int force_passes = opt ? opt->passes : 0;
    const int grid_scale = opt ? opt->grid_scale : 0;
    const int scheme = opt ? opt->scheme : TFFT_SCHEME_BLOCK;
    if (force_passes < 0 || force_passes > 3 || grid_scale < -3 || grid_scale > 3) return TFFT_E_INVALID;
    if (scheme < TFFT_SCHEME_BLOCK || scheme > TFFT_SCHEME_THREAD) return TFFT_E_INVALID;
    // the alternative schemes are not offered for ragged classes
    if (scheme != TFFT_SCHEME_BLOCK && ragged) return TFFT_E_UNSUPPORTED;
    const int k = ilog2_64(n);
    if ((force_passes == 1 && k > TFFT_ONE_PASS_MAX_LOG2) || (force_passes == 2 && (k < 8 || k > 20)) ||
        (force_passes == 3 && k < 12))
        return TFFT_E_UNSUPPORTED;
    p->n = n;
    p->batch = batch;
    p->dtype = dtype;
    p->flags = flags;
    p->kappa = (opt && opt->kappa > 0) ? opt->kappa : (dtype == TFFT_C128 ? TFFT_KAPPA64 : TFFT_KAPPA32);
    p->scheme = scheme;
    p->persistent = (flags & TFFT_PERSISTENT) ? 1 : 0;
    // one pass up to 2^13 (the paper's single-launch limit); two passes up to
    // 2^19 (complex64) / 2^20; three passes above, the shortest first (tiles
    // of the strided passes then hold >= 16 adjacent sub-signals, i.e.
    // >= 128-byte segments per row)
    const int two_max = dtype == TFFT_C128 ? TFFT_TWO_PASS_MAX_LOG2_64 : TFFT_TWO_PASS_MAX_LOG2_32;
    // (the thread-level scheme checks radix-8 butterflies: its one-pass plans
    // stop where the one-pass tile needs a larger thread radix)
    const int one_max = (scheme == TFFT_SCHEME_THREAD && TFFT_ONE_PASS_MAX_LOG2 >= ilog2c(TFFT_E_ROWS_BIG_MIN))
                            ? ilog2c(TFFT_E_ROWS_BIG_MIN) - 1
                            : TFFT_ONE_PASS_MAX_LOG2;
    if (force_passes == 1 && k > one_max) return TFFT_E_UNSUPPORTED;
    const int npass = force_passes ? force_passes : (k <= one_max ? 1 : (k <= two_max ? 2 : 3));
    if (npass == 1) {
        p->passes = 1;
        p->lens[0] = (int)n;
    } else if (npass == 2) {
        // split 1: the longer sub-transform first
        p->passes = 2;
        p->lens[split ? 1 : 0] = 1 << (k / 2);
        p->lens[split ? 0 : 1] = 1 << (k - k / 2);
    } else {
        // split 1: the middle length first
        p->passes = 3;
        const int a = k / 3, b = (k - a) / 2, c = k - a - b;
        p->lens[0] = 1 << (split ? b : a);
        p->lens[1] = 1 << (split ? a : b);
        p->lens[2] = 1 << c;
    }
    if (p->persistent) {
        // the persistent kernel's variants: rows of 64..4096 points, strided
        // and last passes of 64..1024 points
        for (int i = 0; i < p->passes; ++i)
            if (p->lens[i] < 64 || p->lens[i] > (p->passes == 1 ? 4096 : 1024)) return TFFT_E_UNSUPPORTED;
    }
    for (int i = 0; i < p->passes; ++i) {
        const int kind = p->passes == 1 ? KIND_ROWS : (i == p->passes - 1 ? KIND_LAST : KIND_STRIDED);
        const int rc = shape_pass(p, i, p->lens[i], kind, Guser, grid_scale);
        if (rc != TFFT_OK) return rc;
    }
    // multi-pass plans may run their batch in chunks of whole signals, each
    // chunk's passes through one workspace slot
    const int32_t chunk = opt ? opt->chunk : 0;
    if (chunk < 0 || chunk % 64 != 0) return TFFT_E_INVALID;
    p->chunk = (p->passes > 1 && chunk > 0) ? std::min<int64_t>(chunk, batch) : batch;
    p->work_bytes = p->passes > 1 ? (size_t)n * (size_t)p->chunk * esz : 0;
    int64_t cap = 0;
    for (int i = 0; i < p->passes; ++i)  // one-sided multi-pass: one record per sub-signal at most
        cap += p->pass[i].n_groups * ((p->scheme == TFFT_SCHEME_SIGNAL && p->pass[i].kind != KIND_ROWS) ? p->pass[i].G : 1);
    p->rec_cap = std::max<int64_t>(1, cap);
    return TFFT_OK;
}

// Plan construction shared by dense and ragged plans.  host_off (may be
// NULL): element offsets of the `batch` signals inside buffers spanning
// `extent` elements.
int create_plan(tfft_plan *out, int64_t n, int64_t batch, int dtype, const tfft_options *opt, const int64_t *host_off,
                int64_t extent) {
    if (!out) return TFFT_E_INVALID;
    *out = nullptr;
    tfft_plan_s *p = new (std::nothrow) tfft_plan_s();
    if (!p) return TFFT_E_NOMEM;
    int rc = shape_plan(p, n, batch, dtype, opt, host_off != nullptr);
    if (rc != TFFT_OK) {
        delete p;
        return rc;
    }
    (void)hipGetDevice(&p->device);
    p->extent = host_off ? extent : n * batch;
    for (int i = 0; i < p->passes && rc == TFFT_OK; ++i) rc = upload_pass(p, i);
    if (rc == TFFT_OK && p->passes > 1) {
        // w_N^t = lo[t mod 2^b] * hi[t >> b]
        const int k = ilog2_64(n);
        p->itw_bits = (k + 1) / 2;
        const int64_t nlo = int64_t(1) << p->itw_bits, nhi = n >> p->itw_bits;
        std::vector<double> lo(2 * (size_t)nlo), hi(2 * (size_t)nhi);
        for (int64_t t = 0; t < nlo; ++t) {
            const cd w = unit_root(t, n);
            lo[2 * t] = w.real();
            lo[2 * t + 1] = w.imag();
        }
        for (int64_t t = 0; t < nhi; ++t) {
            const cd w = unit_root(t << p->itw_bits, n);
            hi[2 * t] = w.real();
            hi[2 * t + 1] = w.imag();
        }
        rc = upload(&p->d_itw_lo, lo);
        if (rc == TFFT_OK) rc = upload(&p->d_itw_hi, hi);
        if (rc == TFFT_OK && hipMalloc(&p->d_work, p->work_bytes) != hipSuccess) {
            p->d_work = nullptr;
            rc = TFFT_E_NOMEM;
        }
    }
    if (rc == TFFT_OK) {
        if (hipMalloc((void **)&p->d_rep, sizeof(DevReport)) != hipSuccess ||
            hipMalloc((void **)&p->d_recs, sizeof(DevRecord) * (size_t)p->rec_cap) != hipSuccess)
            rc = TFFT_E_NOMEM;
        else if (hipMemset(p->d_rep, 0, sizeof(DevReport)) != hipSuccess)
            rc = TFFT_E_HIP;
    }
    if (rc == TFFT_OK && host_off) {
        std::vector<int64_t> off(host_off, host_off + batch);
        rc = upload(&p->d_sig_off, off);
    }
    if (rc != TFFT_OK) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return TFFT_OK;
}

// A device record as the caller sees it: the group's member mapped back to
// (signal, sub-transform), the residual, threshold and quotient.
tfft_record host_record(const tfft_plan_s *p, const DevRecord &d) {
    tfft_record r;
    std::memset(&r, 0, sizeof(r));
    const bool pass_ok = d.pass >= 0 && d.pass < p->passes;
    const PassPlan &P = p->pass[pass_ok ? d.pass : 0];
    // a member outside the group (never written by the kernels) reads as
    // the group's first signal
    const int mem = (d.member >= 0 && d.member < P.G) ? d.member : 0;
    if (P.kind == KIND_ROWS) {
        r.signal = d.group * P.G + mem;
        r.sub = d.method == TFFT_LOC_THREAD ? (int64_t)d.s : 0;
    } else {
        const int64_t strip = d.group % P.n_strips, ublk = d.group / P.n_strips;
        const int64_t u = ublk * P.rb + mem / P.C, i2 = strip * P.C + mem % P.C;
        if (P.kind == KIND_STRIDED) {
            r.signal = u / P.O;
            r.sub = (u % P.O) * P.S + i2;
        } else {
            r.signal = u;
            r.sub = i2;
        }
    }
    if (r.signal < 0 || r.signal >= p->batch) r.signal = std::min<int64_t>(p->batch - 1, std::max<int64_t>(0, r.signal));
    r.group = d.group;
    r.pass = d.pass;
    r.member = d.member;
    r.action = d.action;
    r.method = d.method;
    r.residual = std::sqrt(d.d1r * d.d1r + d.d1i * d.d1i);
    r.threshold = d.tau;
    const double den = d.d1r * d.d1r + d.d1i * d.d1i;
    r.ratio_re = (d.d2r * d.d1r + d.d2i * d.d1i) / den;
    r.ratio_im = (d.d2i * d.d1r - d.d2r * d.d1i) / den;
    return r;
}

}  // namespace

extern "C" {

int tfft_plan_create_with(tfft_plan *out, int64_t n, int64_t batch, int dtype, const tfft_options *opt) {
    return create_plan(out, n, batch, dtype, opt, nullptr, 0);
}

int tfft_plan_create(tfft_plan *out, int64_t n, int64_t batch, int dtype, uint32_t flags) {
    tfft_options o;
    std::memset(&o, 0, sizeof(o));
    o.flags = flags;
    return tfft_plan_create_with(out, n, batch, dtype, &o);
}

int tfft_plan_destroy(tfft_plan p) {
    free_plan(p);
    return TFFT_OK;
}

int tfft_exec_forward(tfft_plan p, const void *d_in, void *d_out, int ft_mode, void *hip_stream) {
    return exec(p, d_in, d_out, ft_mode, hip_stream, false);
}

int tfft_exec_inverse(tfft_plan p, const void *d_in, void *d_out, int ft_mode, void *hip_stream) {
    return exec(p, d_in, d_out, ft_mode, hip_stream, true);
}

// The same execution with its report and workspace in the static scratch:
// [report counters | records | workspace], each part 256-byte aligned.  No
// allocation of any kind; the counters are cleared by the reset kernel of
// the execution itself.
int tfft_exec_noalloc(tfft_plan p, const void *d_in, void *d_out, int ft_mode, int inverse, void *hip_stream) {
    if (!p) return TFFT_E_INVALID;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t rep_bytes = up(sizeof(DevReport));
    const size_t rec_bytes = up(sizeof(DevRecord) * (size_t)p->rec_cap);
    const size_t work_bytes = p->passes > 1 ? up(p->work_bytes) : 0;
    if (rep_bytes + rec_bytes + work_bytes > kScratchBytes) return TFFT_E_SCRATCH;
    Guard guard(p->device);
    unsigned char *base = static_cast<unsigned char *>(scratch_address(p->device));
    if (!base) return TFFT_E_HIP;
    const ExecBufs b{reinterpret_cast<DevReport *>(base), reinterpret_cast<DevRecord *>(base + rep_bytes),
                     work_bytes ? base + rep_bytes + rec_bytes : nullptr};
    return exec(p, d_in, d_out, ft_mode, hip_stream, inverse != 0, &b);
}

int tfft_get_report(tfft_plan p, tfft_counts *counts, tfft_record *recs, int64_t cap) {
    if (!p || cap < 0 || (cap > 0 && !recs)) return TFFT_E_INVALID;
    if (!p->executed) return TFFT_E_STATE;
    Guard guard(p->device);
    if (hipStreamSynchronize(p->last_stream) != hipSuccess) return TFFT_E_HIP;
    DevReport h;
    if (hipMemcpy(&h, p->rep_last, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return TFFT_E_HIP;
    const int64_t nrec = std::min<int64_t>((int64_t)h.n_flag, p->rec_cap);
    std::vector<DevRecord> dr((size_t)nrec);
    if (nrec > 0 &&
        hipMemcpy(dr.data(), p->recs_last, sizeof(DevRecord) * (size_t)nrec, hipMemcpyDeviceToHost) != hipSuccess)
        return TFFT_E_HIP;
    int64_t groups = 0;
    if (p->last_mode != TFFT_FT_OFF)
        for (int i = 0; i < p->passes; ++i)  // one-sided: every (sub-)signal is checked
            groups += p->pass[i].n_groups * ((p->scheme == TFFT_SCHEME_SIGNAL && p->pass[i].kind != KIND_ROWS) ? p->pass[i].G : 1);
    if (counts) {
        counts->groups_checked = groups;
        counts->detected = (int64_t)h.n_flag;
        counts->corrected = (int64_t)h.corrected;
        counts->uncorrectable = (int64_t)h.uncorrectable;
        counts->benign = (int64_t)h.benign;
        counts->n_records = nrec;
        counts->dropped = (int64_t)h.n_flag - nrec;
    }
    std::vector<tfft_record> out((size_t)nrec);
    for (int64_t i = 0; i < nrec; ++i) out[(size_t)i] = host_record(p, dr[(size_t)i]);
    // deterministic order whatever the order the device wrote them in
    std::sort(out.begin(), out.end(), [](const tfft_record &x, const tfft_record &y) {
        if (x.signal != y.signal) return x.signal < y.signal;
        if (x.pass != y.pass) return x.pass < y.pass;
        if (x.group != y.group) return x.group < y.group;
        return x.sub < y.sub;
    });
    for (int64_t i = 0; i < std::min(cap, nrec); ++i) recs[i] = out[(size_t)i];
    const bool bad = h.uncorrectable > 0 || (p->last_mode == TFFT_FT_CORRECT && (int64_t)h.n_flag > nrec);
    return bad ? TFFT_UNCORRECTABLE : TFFT_OK;
}

int tfft_set_faults(tfft_plan p, const tfft_fault *specs, int64_t n) {
    if (!p || n < 0 || (n > 0 && !specs)) return TFFT_E_INVALID;
    Guard guard(p->device);
    // the fault tables are replaced: wait for the last execution that may read them
    if (p->executed && hipStreamSynchronize(p->last_stream) != hipSuccess) return TFFT_E_HIP;
    clear_faults(p);
    if (n == 0) return TFFT_OK;
    std::vector<std::vector<DevFault>> per(p->passes);
    for (int64_t f = 0; f < n; ++f) {
        const tfft_fault &s = specs[f];
        if (s.signal < 0 || s.signal >= p->batch || s.pass < 0 || s.pass >= p->passes) return TFFT_E_INVALID;
        if (s.index < 0 || s.index >= p->n) return TFFT_E_INVALID;
        if (s.mode < TFFT_FAULT_ADD || s.mode > TFFT_FAULT_FLIP_IM) return TFFT_E_INVALID;
        if (s.mode != TFFT_FAULT_ADD && (s.bit < 0 || s.bit >= (p->dtype == TFFT_C128 ? 64 : 32)))
            return TFFT_E_INVALID;
        const PassPlan &P = p->pass[s.pass];
        if (s.stage < -1 || s.stage >= P.stages) return TFFT_E_INVALID;
        const int M = P.M, E = P.E, T = M / E;
        int64_t g, pos;
        int b;
        if (P.kind == KIND_ROWS) {
            g = s.signal / P.G;
            b = (int)(s.signal % P.G);
            pos = s.index;
        } else {
            const int64_t sub = s.index / M;
            pos = s.index % M;
            int64_t u, i;
            if (P.kind == KIND_STRIDED) {
                u = s.signal * P.O + sub / P.S;
                i = sub % P.S;
            } else {
                u = s.signal;
                i = sub;
            }
            g = (u / P.rb) * P.n_strips + i / P.C;
            b = (int)((u % P.rb) * P.C + i % P.C);
        }
        DevFault d;
        std::memset(&d, 0, sizeof(d));
        d.group = g;
        d.member = b;
        d.stage = s.stage;
        d.dre = s.mode == TFFT_FAULT_ADD ? s.dre : 0.0;
        d.dim = s.mode == TFFT_FAULT_ADD ? s.dim : 0.0;
        d.mode = s.mode;
        d.bit = s.bit;
        if (s.stage < 0) {
            d.j = (int)(pos % T);
            d.m = (int)(pos / T);
        } else {
            const int RAD = stage_radix(M, E, s.stage), NS = stage_ns(M, E, s.stage), NB = E / RAD;
            const int64_t q = (pos / NS) % RAD;
            const int64_t i = (pos / ((int64_t)NS * RAD)) * NS + pos % NS;
            d.j = (int)(i % T);
            d.m = (int)(i / T + q * NB);
        }
        per[s.pass].push_back(d);
    }
    for (int i = 0; i < p->passes; ++i) {
        auto &v = per[i];
        if (v.empty()) continue;
        PassPlan &P = p->pass[i];
        std::stable_sort(v.begin(), v.end(), [](const DevFault &x, const DevFault &y) { return x.group < y.group; });
        std::vector<int32_t> head((size_t)P.n_groups, -1);
        for (size_t k = 0; k < v.size(); ++k) {
            v[k].next = (k + 1 < v.size() && v[k + 1].group == v[k].group) ? (int32_t)(k + 1) : -1;
            if (k == 0 || v[k - 1].group != v[k].group) head[(size_t)v[k].group] = (int32_t)k;
        }
        int rc = upload(&P.d_fault_head, head);
        if (rc == TFFT_OK) rc = upload(&P.d_faults, v);
        if (rc != TFFT_OK) {
            clear_faults(p);
            return rc;
        }
    }
    p->nfaults = n;
    return TFFT_OK;
}

int tfft_set_timing(tfft_plan p, int enable) {
    if (!p) return TFFT_E_INVALID;
    Guard guard(p->device);
    if (enable) {
        for (auto &e : p->ev)
            if (!e && hipEventCreate(&e) != hipSuccess) return TFFT_E_HIP;
    }
    p->timing = enable ? 1 : 0;
    return TFFT_OK;
}

int tfft_get_timings(tfft_plan p, double *pass_ms, double *correct_ms) {
    if (!p) return TFFT_E_INVALID;
    if (!p->executed || !p->timed_last) return TFFT_E_STATE;
    Guard guard(p->device);
    if (hipEventSynchronize(p->ev[2 * p->passes]) != hipSuccess) return TFFT_E_HIP;
    if (p->timed_last == 2) {
        // chunked execution: the passes of the chunks interleave; the whole
        // execution is reported as pass 0
        float a = 0.f;
        if (hipEventElapsedTime(&a, p->ev[0], p->ev[2 * p->passes]) != hipSuccess) return TFFT_E_HIP;
        for (int i = 0; i < kMaxPasses; ++i) {
            if (pass_ms) pass_ms[i] = i == 0 ? a : 0.0;
            if (correct_ms) correct_ms[i] = 0.0;
        }
        return TFFT_OK;
    }
    for (int i = 0; i < kMaxPasses; ++i) {
        float a = 0.f, b = 0.f;
        if (i < p->passes) {
            if (hipEventElapsedTime(&a, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess) return TFFT_E_HIP;
            if (hipEventElapsedTime(&b, p->ev[2 * i + 1], p->ev[2 * i + 2]) != hipSuccess) return TFFT_E_HIP;
        }
        if (pass_ms) pass_ms[i] = a;
        if (correct_ms) correct_ms[i] = p->launched_correct ? b : 0.0;
    }
    return TFFT_OK;
}

}  // extern "C"

struct tfft_ragged_s {
    int device = 0;
    int dtype = 0;
    tfft_options opt{};
    int64_t count = 0, extent = 0;
    std::vector<int64_t> lengths, offsets;
    struct Class {
        int64_t n = 0;
        std::vector<int64_t> members;  // ragged indices of its signals
        tfft_plan plan = nullptr;
    };
    std::vector<Class> classes;
    std::vector<int64_t> class_of, local_of;
    // captured graph and its key
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *g_in = nullptr;
    void *g_out = nullptr;
    int g_mode = -1, g_inv = -1;
    hipStream_t g_stream = nullptr;
    hipStream_t last_stream = nullptr;
    int executed = 0, last_mode = 0;
    // parallel branches of the captured graph: classes are independent, so
    // they are captured on TFFT_GRAPH_BRANCHES forked streams and joined
    hipStream_t aux[TFFT_GRAPH_BRANCHES] = {};
    hipEvent_t ev_fork = nullptr, ev_join[TFFT_GRAPH_BRANCHES] = {};
    std::vector<int> branch_of;  // class -> branch
    std::vector<std::vector<tfft_fault>> class_faults;  // installed faults per class (class-local signals)

    // persistent execution (TFFT_PERSISTENT): one kernel drains a queue of
    // work items covering every pass of every class
    int persistent = 0;
    int64_t item_tiles = 0;               // target tiles per work item (0: default)
    int item_interleave = 0;              // items of a chunk take every n-th group (1) or a range (0)
    int n_queues = kPQueues;              // work queues (one per XCD, or 1)
    int chunk_div = 8;                    // dependency chunks per class, about
    int64_t *d_qbeg = nullptr;            // queue bounds, n_queues + 1
    std::vector<int> task_class, task_pass;
    std::vector<PItem> h_items;
    int n_done = 0;                       // release counters: one per (task, chunk)
    PItem *d_items = nullptr;
    PTask *d_tasks = nullptr;
    int32_t *d_need = nullptr, *d_done = nullptr, *d_err = nullptr;
    unsigned long long *d_head = nullptr;
    DevReport *d_rep = nullptr;           // one report for all classes
    DevRecord *d_recs = nullptr;
    int64_t rec_cap = 0;
    int tasks_valid = 0;                  // d_tasks holds the tables for this key:
    const void *t_in = nullptr;
    void *t_out = nullptr;
    int t_mode = -1, t_inv = -1;
};

namespace {

void drop_graph(tfft_ragged_s *r) {
    if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    r->gexec = nullptr;
    r->graph = nullptr;
    r->g_in = nullptr;
    r->g_out = nullptr;
}

int build_class(tfft_ragged_s *r, size_t ci, const tfft_options &opt) {
    auto &C = r->classes[ci];
    std::vector<int64_t> off;
    off.reserve(C.members.size());
    for (int64_t i : C.members) off.push_back(r->offsets[(size_t)i]);
    tfft_plan np = nullptr;
    const int rc = create_plan(&np, C.n, (int64_t)C.members.size(), r->dtype, &opt, off.data(), r->extent);
    if (rc != TFFT_OK) return rc;
    if (C.plan) tfft_plan_destroy(C.plan);
    C.plan = np;
    return TFFT_OK;
}

int ragged_launch(tfft_ragged_s *r, const void *d_in, void *d_out, int ft_mode, int inverse, hipStream_t st) {
    for (auto &C : r->classes) {
        const int rc = exec(C.plan, d_in, d_out, ft_mode, st, inverse != 0);
        if (rc != TFFT_OK) return rc;
    }
    return TFFT_OK;
}

// Balance the classes over the branches by bytes (largest first, each to the
// least loaded branch).
void assign_branches(tfft_ragged_s *r) {
    const size_t nc = r->classes.size();
    std::vector<size_t> order(nc);
    for (size_t c = 0; c < nc; ++c) order[c] = c;
    auto bytes = [&](size_t c) { return r->classes[c].n * (int64_t)r->classes[c].members.size(); };
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return bytes(a) > bytes(b); });
    int64_t load[TFFT_GRAPH_BRANCHES] = {};
    r->branch_of.assign(nc, 0);
    for (size_t c : order) {
        int b = 0;
        for (int q = 1; q < TFFT_GRAPH_BRANCHES; ++q)
            if (load[q] < load[b]) b = q;
        r->branch_of[c] = b;
        load[b] += bytes(c);
    }
}

// Launch every class on its branch, forked from and joined back into st
// (used under stream capture, where it records a graph with parallel
// branches).
int ragged_launch_branches(tfft_ragged_s *r, const void *d_in, void *d_out, int ft_mode, int inverse,
                           hipStream_t st) {
    if (!r->ev_fork) {
        if (hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming) != hipSuccess) return TFFT_E_HIP;
        for (int b = 0; b < TFFT_GRAPH_BRANCHES; ++b)
            if (hipStreamCreateWithFlags(&r->aux[b], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&r->ev_join[b], hipEventDisableTiming) != hipSuccess)
                return TFFT_E_HIP;
        assign_branches(r);
    }
    const int nb = (int)std::min<size_t>(TFFT_GRAPH_BRANCHES, r->classes.size());
    if (hipEventRecord(r->ev_fork, st) != hipSuccess) return TFFT_E_HIP;
    for (int b = 0; b < nb; ++b)
        if (hipStreamWaitEvent(r->aux[b], r->ev_fork, 0) != hipSuccess) return TFFT_E_HIP;
    int rc = TFFT_OK;
    for (size_t c = 0; c < r->classes.size() && rc == TFFT_OK; ++c)
        rc = exec(r->classes[c].plan, d_in, d_out, ft_mode, r->aux[r->branch_of[c] % nb], inverse != 0);
    // join every forked branch, also after a failure, so that the capture ends cleanly
    for (int b = 0; b < nb; ++b)
        if (hipEventRecord(r->ev_join[b], r->aux[b]) != hipSuccess || hipStreamWaitEvent(st, r->ev_join[b], 0) != hipSuccess)
            rc = TFFT_E_HIP;
    return rc;
}

constexpr int64_t kPItemTiles = 32;  // default tiles per work item

// Signals per dependency chunk of a class: a multiple of the signals every
// pass's checksum group spans (so that no group straddles two chunks), at
// most 64, and otherwise small enough for about `div` chunks per class (so
// that a later pass starts on the first chunks while the last ones are still
// in the previous pass).
int64_t class_chunk(const tfft_plan_s *p, int div) {
    int64_t span = 1;
    for (int i = 0; i < p->passes; ++i) {
        const PassPlan &P = p->pass[i];
        const int64_t s = P.kind == KIND_ROWS ? P.G : (P.kind == KIND_STRIDED ? (P.rb + P.O - 1) / P.O : P.rb);
        span = std::max(span, s);
    }
    int64_t q = 64;
    while (q > span && q * div > p->batch) q /= 2;
    return std::max(q, span);
}

void persist_free(tfft_ragged_s *r) {
    (void)hipFree(r->d_items);
    (void)hipFree(r->d_tasks);
    (void)hipFree(r->d_need);
    (void)hipFree(r->d_done);
    (void)hipFree(r->d_err);
    (void)hipFree(r->d_head);
    (void)hipFree(r->d_qbeg);
    r->d_qbeg = nullptr;
    (void)hipFree(r->d_rep);
    (void)hipFree(r->d_recs);
    r->d_items = nullptr;
    r->d_tasks = nullptr;
    r->d_need = r->d_done = r->d_err = nullptr;
    r->d_head = nullptr;
    r->d_rep = nullptr;
    r->d_recs = nullptr;
    r->tasks_valid = 0;
}

// The work queue of a persistent ragged plan from its class plans: tasks
// (class, pass), chunks of signals per class (class_chunk), items of up to
// kPSlotCap groups (about a target number of tiles each), and the items per
// (task, chunk) that a later pass waits for.  Queue order: every multi-pass class's pass 0, then
// pass 1, then pass 2 (larger classes first within a level), then the
// one-pass classes, whose items need nothing and fill the end.
int persist_build(tfft_ragged_s *r) {
    persist_free(r);
    r->task_class.clear();
    r->task_pass.clear();
    const size_t nc = r->classes.size();
    std::vector<int> task0(nc);
    for (size_t c = 0; c < nc; ++c) {
        task0[c] = (int)r->task_class.size();
        for (int i = 0; i < r->classes[c].plan->passes; ++i) {
            r->task_class.push_back((int)c);
            r->task_pass.push_back(i);
        }
    }
    const int ntask = (int)r->task_class.size();
    std::vector<int> done_base(ntask);
    int nd = 0;
    for (int t = 0; t < ntask; ++t) {
        done_base[t] = nd;
        const tfft_plan_s *pc = r->classes[(size_t)r->task_class[t]].plan;
        const int64_t q = class_chunk(pc, r->chunk_div);
        nd += (int)((pc->batch + q - 1) / q);
    }
    r->n_done = nd;
    std::vector<int32_t> need((size_t)std::max(1, nd), 0);
    // tiles per item: as tuned, else 32 (an item's start, with its first
    // load not overlapped, then costs a few percent of its work); items keep
    // whole groups, at most kPSlotCap of them
    const int64_t target = r->item_tiles > 0 ? r->item_tiles : kPItemTiles;
    // items per task, in chunk order
    std::vector<std::vector<PItem>> per(ntask);
    for (int t = 0; t < ntask; ++t) {
        const tfft_plan_s *p = r->classes[(size_t)r->task_class[t]].plan;
        const PassPlan &P = p->pass[r->task_pass[t]];
        const int64_t rounds = std::max(1, P.G / std::max(1, P.C));  // tiles per group
        const int64_t K = std::max<int64_t>(1, std::min<int64_t>(kPSlotCap, target / rounds));
        const int64_t Q = class_chunk(p, r->chunk_div);
        for (int64_t q = 0; q * Q < p->batch; ++q) {
            const ChunkGeom cg = chunk_geom(p, P, q * Q, std::min(Q, p->batch - q * Q));
            const int64_t n_it = (cg.n_groups + K - 1) / K;
            for (int64_t i = 0; i < n_it; ++i) {
                PItem it;
                it.task = t;
                it.chunk = (int32_t)q;
                if (r->item_interleave) {
                    // item i takes groups i, i + n_it, ...: the workgroups
                    // running the chunk's items side by side work on
                    // neighbouring strips at the same time
                    it.g0 = cg.g_base + i;
                    it.g1 = cg.g_base + cg.n_groups;
                    it.step = n_it;
                } else {
                    it.g0 = cg.g_base + i * K;
                    it.g1 = std::min(it.g0 + K, cg.g_base + cg.n_groups);
                    it.step = 1;
                }
                per[t].push_back(it);
                ++need[(size_t)(done_base[t] + q)];
            }
        }
    }
    // classes by bytes, largest first
    std::vector<size_t> order(nc);
    for (size_t c = 0; c < nc; ++c) order[c] = c;
    auto bytes = [&](size_t c) { return r->classes[c].n * (int64_t)r->classes[c].members.size(); };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return bytes(a) > bytes(b); });
    // Chunks to queues: every item of a chunk (all its passes) in one queue,
    // so that a wait never crosses queues; the chunks, largest first, each to
    // the queue with the fewest bytes so far.
    const int nq = std::max(1, std::min(kPQueues, r->n_queues));
    std::vector<std::vector<int>> qof(nc);
    {
        struct Ck {
            size_t c;
            int64_t q, bytes;
        };
        std::vector<Ck> cks;
        for (size_t c = 0; c < nc; ++c) {
            const tfft_plan_s *p = r->classes[c].plan;
            const int64_t Q = class_chunk(p, r->chunk_div);
            qof[c].assign((size_t)((p->batch + Q - 1) / Q), 0);
            for (int64_t q = 0; q * Q < p->batch; ++q)
                cks.push_back({c, q, std::min(Q, p->batch - q * Q) * r->classes[c].n * p->passes});
        }
        std::stable_sort(cks.begin(), cks.end(), [](const Ck &a, const Ck &b) { return a.bytes > b.bytes; });
        std::vector<int64_t> load((size_t)nq, 0);
        for (const Ck &k : cks) {
            const size_t best = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            qof[k.c][(size_t)k.q] = (int)best;
            load[best] += k.bytes;
        }
    }
    // each queue in level order: pass 0 of its multi-pass chunks (larger
    // classes first), then pass 1, then pass 2, then its one-pass chunks
    r->h_items.clear();
    std::vector<int64_t> qbeg((size_t)kPQueues + 1, 0);
    for (int k = 0; k < nq; ++k) {
        qbeg[(size_t)k] = (int64_t)r->h_items.size();
        for (int level = 0; level < kMaxPasses; ++level)
            for (size_t c : order)
                if (r->classes[c].plan->passes > 1 && level < r->classes[c].plan->passes)
                    for (const PItem &it : per[(size_t)(task0[c] + level)])
                        if (qof[c][(size_t)it.chunk] == k) r->h_items.push_back(it);
        for (size_t c : order)
            if (r->classes[c].plan->passes == 1)
                for (const PItem &it : per[(size_t)task0[c]])
                    if (qof[c][(size_t)it.chunk] == k) r->h_items.push_back(it);
    }
    for (int k = nq; k <= kPQueues; ++k) qbeg[(size_t)k] = (int64_t)r->h_items.size();
    r->rec_cap = 0;
    for (auto &C : r->classes) r->rec_cap += C.plan->rec_cap;
    int rc = upload(&r->d_items, r->h_items);
    if (rc == TFFT_OK) rc = upload(&r->d_need, need);
    if (rc == TFFT_OK) rc = upload(&r->d_qbeg, qbeg);
    if (rc == TFFT_OK && (hipMalloc((void **)&r->d_tasks, sizeof(PTask) * (size_t)std::max(1, ntask)) != hipSuccess ||
                          hipMalloc((void **)&r->d_done, sizeof(int32_t) * (size_t)std::max(1, nd)) != hipSuccess ||
                          hipMalloc((void **)&r->d_err, sizeof(int32_t)) != hipSuccess ||
                          hipMalloc((void **)&r->d_head, sizeof(unsigned long long) * kPQueues) != hipSuccess ||
                          hipMalloc((void **)&r->d_rep, sizeof(DevReport)) != hipSuccess ||
                          hipMalloc((void **)&r->d_recs, sizeof(DevRecord) * (size_t)r->rec_cap) != hipSuccess))
        rc = TFFT_E_NOMEM;
    if (rc != TFFT_OK) persist_free(r);
    return rc;
}

// The task table for one execution (buffers, direction, mode), uploaded when
// any of them changed (a synchronous copy: never under stream capture).
int persist_tasks(tfft_ragged_s *r, const void *d_in, void *d_out, int mode, int inverse) {
    if (r->tasks_valid && r->t_in == d_in && r->t_out == d_out && r->t_mode == mode && r->t_inv == inverse)
        return TFFT_OK;
    const int ntask = (int)r->task_class.size();
    std::vector<PTask> tasks((size_t)ntask);
    int nd = 0;
    for (int t = 0; t < ntask; ++t) {
        const tfft_plan_s *p = r->classes[(size_t)r->task_class[t]].plan;
        const int i = r->task_pass[t];
        const ChunkGeom cg = chunk_geom(p, p->pass[i], 0, p->batch);
        PTask &k = tasks[(size_t)t];
        std::memset(&k, 0, sizeof(k));
        k.a = pass_args(p, i, cg, p->batch, d_in, d_out, p->d_work, p->d_sig_off, inverse != 0, mode, r->d_rep,
                        r->d_recs);
        k.a.rec_cap = r->rec_cap;
        k.a.task = t;
        k.variant = pvariant_id(p->pass[i].kind, p->pass[i].M);
        k.dep = i > 0 ? t - 1 : -1;
        k.done_base = nd;
        k.fix = mode == TFFT_FT_CORRECT;
        k.publish = i + 1 < p->passes;
        nd += (int)((p->batch + class_chunk(p, r->chunk_div) - 1) / class_chunk(p, r->chunk_div));
    }
    if (hipMemcpy(r->d_tasks, tasks.data(), sizeof(PTask) * (size_t)ntask, hipMemcpyHostToDevice) != hipSuccess)
        return TFFT_E_HIP;
    r->tasks_valid = 1;
    r->t_in = d_in;
    r->t_out = d_out;
    r->t_mode = mode;
    r->t_inv = inverse;
    return TFFT_OK;
}

// One persistent execution on st: the queue reset and the kernel.
int persist_launch_all(tfft_ragged_s *r, int mode, hipStream_t st) {
    PQueue q;
    q.items = r->d_items;
    q.n_items = (int64_t)r->h_items.size();
    q.tasks = r->d_tasks;
    q.head = r->d_head;
    q.q_begin = r->d_qbeg;
    q.n_queues = std::max(1, std::min(kPQueues, r->n_queues));
    q.pad_ = 0;
    q.done = r->d_done;
    q.need = r->d_need;
    q.err = r->d_err;
    q.spin_limit = int64_t(1) << 21;  // a few seconds of polls at most
    const int fp64 = r->dtype == TFFT_C128, ft = mode != TFFT_FT_OFF;
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device);
    const int occ = std::max(1, persist_occupancy(fp64, ft));
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(q.n_items, (int64_t)occ * std::max(1, cus)));
    if (launch_persist_reset(q, r->n_done, r->d_rep, st) != hipSuccess) return TFFT_E_HIP;
    if (launch_persist(fp64, ft, q, grid, st) != hipSuccess) return TFFT_E_HIP;
    return TFFT_OK;
}

// Autotuner of a persistent ragged plan: coordinate descent over the
// classes (largest first) on the time of the whole persistent execution
// (FT CORRECT on the caller's buffers): per class the pass count, the split
// of the stages over the passes and the checksum group size (one-pass classes
// keep one pass), then the tiles per work item.
int persist_tune(tfft_ragged_s *r, const void *d_in, void *d_out, hipStream_t st, int reps) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TFFT_E_HIP;
    auto time_all = [&](float *ms) -> int {
        drop_graph(r);
        int rc = persist_tasks(r, d_in, d_out, TFFT_FT_CORRECT, 0);
        for (int t = 0; t <= reps && rc == TFFT_OK; ++t) {  // the first run warms up
            if (t == 1 && hipEventRecord(e0, st) != hipSuccess) rc = TFFT_E_HIP;
            if (rc == TFFT_OK) rc = persist_launch_all(r, TFFT_FT_CORRECT, st);
        }
        if (rc == TFFT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(ms, e0, e1) != hipSuccess))
            rc = TFFT_E_HIP;
        return rc;
    };
    std::vector<tfft_options> cur(r->classes.size(), r->opt);
    float best = 0.f;
    int status = time_all(&best);
    std::vector<size_t> order(r->classes.size());
    for (size_t c = 0; c < order.size(); ++c) order[c] = c;
    auto bytes = [&](size_t c) { return r->classes[c].n * (int64_t)r->classes[c].members.size(); };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return bytes(a) > bytes(b); });
    for (size_t ci : order) {
        if (status != TFFT_OK) break;
        const int k = ilog2_64(r->classes[ci].n);
        std::vector<tfft_options> cand;
        if (k <= TFFT_ONE_PASS_MAX_LOG2) {
            for (int grp : {0, 16, 32, 64}) {
                tfft_options o = r->opt;
                o.passes = 1;
                o.group = grp;
                cand.push_back(o);
            }
        } else {
            for (int ps = 2; ps <= 3; ++ps)
                for (int sp = 0; sp <= 1; ++sp)
                    for (int grp : {0, 16}) {
                        if ((ps == 2 && k > 20) || (ps == 3 && k < 12)) continue;
                        tfft_options o = r->opt;
                        o.passes = ps;
                        o.split = sp;
                        o.group = grp;
                        cand.push_back(o);
                    }
        }
        tfft_options best_o = cur[ci];
        for (const auto &o : cand) {
            if (build_class(r, ci, o) != TFFT_OK) continue;  // unsupported candidate
            float ms = 0.f;
            if (persist_build(r) != TFFT_OK || time_all(&ms) != TFFT_OK) continue;
            if (ms < best) {
                best = ms;
                best_o = o;
            }
        }
        cur[ci] = best_o;
        status = build_class(r, ci, best_o);
        if (status == TFFT_OK) status = persist_build(r);
    }
    // The layout of the queue, one parameter at a time, each against a fresh
    // measurement of every candidate (the current value among them): tiles
    // per work item, item layout (range or interleaved), queues (one per XCD
    // or one), dependency chunks per class (about 8 or about 32).
    auto pick = [&](const std::vector<int64_t> &cands, const std::function<void(int64_t)> &set) {
        int64_t bestv = cands.front();
        float bestms = 3.4e38f;
        for (int64_t v : cands) {
            if (status != TFFT_OK) break;
            set(v);
            float ms = 0.f;
            if (persist_build(r) == TFFT_OK && time_all(&ms) == TFFT_OK && ms < bestms) {
                bestms = ms;
                bestv = v;
            }
        }
        set(bestv);
    };
    pick({8, 16, 32, 64, 128}, [&](int64_t v) { r->item_tiles = v; });
    pick({0, 1}, [&](int64_t v) { r->item_interleave = (int)v; });
    pick({1, kPQueues}, [&](int64_t v) { r->n_queues = (int)v; });
    pick({8, 32}, [&](int64_t v) { r->chunk_div = (int)v; });
    if (status == TFFT_OK) status = persist_build(r);
    // the new class plans get the faults installed on the old ones
    for (size_t ci = 0; ci < r->classes.size() && status == TFFT_OK; ++ci)
        if (ci < r->class_faults.size() && !r->class_faults[ci].empty())
            status = tfft_set_faults(r->classes[ci].plan, r->class_faults[ci].data(),
                                     (int64_t)r->class_faults[ci].size());
    r->tasks_valid = 0;
    drop_graph(r);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

}  // namespace

extern "C" {

int tfft_ragged_create(tfft_ragged *out, int64_t count, const int64_t *lengths, const int64_t *offsets, int dtype,
                       const tfft_options *opt) {
    if (!out) return TFFT_E_INVALID;
    *out = nullptr;
    if (count < 1 || !lengths || !offsets || dtype < TFFT_C64 || dtype > TFFT_C128) return TFFT_E_INVALID;
    int64_t extent = 0;
    std::vector<std::pair<int64_t, int64_t>> spans((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const int64_t n = lengths[i], o = offsets[i];
        if (n < 2 || n > (int64_t(1) << 24) || (n & (n - 1)) != 0 || o < 0 || o > (int64_t(1) << 40))
            return TFFT_E_INVALID;
        spans[(size_t)i] = {o, o + n};
        extent = std::max(extent, o + n);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return TFFT_E_INVALID;  // signals overlap
    tfft_ragged_s *r = new (std::nothrow) tfft_ragged_s();
    if (!r) return TFFT_E_NOMEM;
    (void)hipGetDevice(&r->device);
    r->dtype = dtype;
    if (opt) r->opt = *opt;
    r->count = count;
    r->extent = extent;
    r->lengths.assign(lengths, lengths + count);
    r->offsets.assign(offsets, offsets + count);
    r->class_of.resize((size_t)count);
    r->local_of.resize((size_t)count);
    std::vector<int64_t> ns(r->lengths);
    std::sort(ns.begin(), ns.end());
    ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
    r->classes.resize(ns.size());
    for (size_t c = 0; c < ns.size(); ++c) r->classes[c].n = ns[c];
    for (int64_t i = 0; i < count; ++i) {
        const size_t c = (size_t)(std::lower_bound(ns.begin(), ns.end(), r->lengths[(size_t)i]) - ns.begin());
        r->class_of[(size_t)i] = (int64_t)c;
        r->local_of[(size_t)i] = (int64_t)r->classes[c].members.size();
        r->classes[c].members.push_back(i);
    }
    r->persistent = (r->opt.flags & TFFT_PERSISTENT) ? 1 : 0;
    r->item_interleave = (r->opt.flags & TFFT_PERSIST_INTERLEAVE) ? 1 : 0;
    r->n_queues = (r->opt.flags & TFFT_PERSIST_ONE_QUEUE) ? 1 : kPQueues;
    for (size_t c = 0; c < r->classes.size(); ++c) {
        const int rc = build_class(r, c, r->opt);
        if (rc != TFFT_OK) {
            tfft_ragged_destroy(r);
            return rc;
        }
    }
    if (r->persistent) {
        const int rc = persist_build(r);
        if (rc != TFFT_OK) {
            tfft_ragged_destroy(r);
            return rc;
        }
    }
    *out = r;
    return TFFT_OK;
}

int tfft_ragged_destroy(tfft_ragged r) {
    if (!r) return TFFT_OK;
    Guard guard(r->device);
    drop_graph(r);
    persist_free(r);
    for (auto &C : r->classes) tfft_plan_destroy(C.plan);
    for (int b = 0; b < TFFT_GRAPH_BRANCHES; ++b) {
        if (r->aux[b]) (void)hipStreamDestroy(r->aux[b]);
        if (r->ev_join[b]) (void)hipEventDestroy(r->ev_join[b]);
    }
    if (r->ev_fork) (void)hipEventDestroy(r->ev_fork);
    delete r;
    return TFFT_OK;
}

int tfft_ragged_exec(tfft_ragged r, const void *d_in, void *d_out, int ft_mode, int inverse, int use_graph,
                     void *hip_stream) {
    if (!r || !d_in || !d_out) return TFFT_E_INVALID;
    if (use_graph && !hip_stream) return TFFT_E_INVALID;
    Guard guard(r->device);
    hipStream_t st = (hipStream_t)hip_stream;
    int rc;
    if (r->persistent) {
        if (ft_mode < TFFT_FT_OFF || ft_mode > TFFT_FT_CORRECT) return TFFT_E_INVALID;
        if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 15)) return TFFT_E_INVALID;
        const size_t bytes = (size_t)r->extent * (r->dtype == TFFT_C128 ? 16 : 8);
        const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
        if ((a < b ? b - a : a - b) < bytes) return TFFT_E_INVALID;  // in place or overlapping
        if ((rc = persist_tasks(r, d_in, d_out, ft_mode, inverse)) != TFFT_OK) return rc;
        if (!use_graph) {
            rc = persist_launch_all(r, ft_mode, st);
        } else {
            if (!(r->gexec && r->g_in == d_in && r->g_out == d_out && r->g_mode == ft_mode && r->g_inv == inverse &&
                  r->g_stream == st)) {
                drop_graph(r);
                if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return TFFT_E_HIP;
                rc = persist_launch_all(r, ft_mode, st);
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(st, &g);
                if (rc != TFFT_OK || e != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc != TFFT_OK ? rc : TFFT_E_HIP;
                }
                r->graph = g;
                if (hipGraphInstantiate(&r->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
                    drop_graph(r);
                    return TFFT_E_HIP;
                }
                r->g_in = d_in;
                r->g_out = d_out;
                r->g_mode = ft_mode;
                r->g_inv = inverse;
                r->g_stream = st;
            }
            rc = hipGraphLaunch(r->gexec, st) == hipSuccess ? TFFT_OK : TFFT_E_HIP;
        }
        if (rc == TFFT_OK) {
            r->executed = 1;
            r->last_mode = ft_mode;
            r->last_stream = st;
        }
        return rc;
    }
    if (!use_graph) {
        rc = ragged_launch(r, d_in, d_out, ft_mode, inverse, st);
    } else {
        if (!(r->gexec && r->g_in == d_in && r->g_out == d_out && r->g_mode == ft_mode && r->g_inv == inverse &&
              r->g_stream == st)) {
            drop_graph(r);
            for (auto &C : r->classes) C.plan->timing = 0;  // no event nodes in the graph
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return TFFT_E_HIP;
            rc = ragged_launch_branches(r, d_in, d_out, ft_mode, inverse, st);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(st, &g);
            if (rc != TFFT_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return rc != TFFT_OK ? rc : TFFT_E_HIP;
            }
            r->graph = g;
            if (hipGraphInstantiate(&r->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(r);
                return TFFT_E_HIP;
            }
            r->g_in = d_in;
            r->g_out = d_out;
            r->g_mode = ft_mode;
            r->g_inv = inverse;
            r->g_stream = st;
        }
        rc = hipGraphLaunch(r->gexec, st) == hipSuccess ? TFFT_OK : TFFT_E_HIP;
        for (auto &C : r->classes) {
            C.plan->executed = 1;
            C.plan->last_mode = ft_mode;
            C.plan->last_stream = st;
            C.plan->timed_last = 0;
            C.plan->launched_correct = ft_mode == TFFT_FT_CORRECT;
        }
    }
    if (rc == TFFT_OK) {
        r->executed = 1;
        r->last_mode = ft_mode;
        r->last_stream = st;
    }
    return rc;
}

int tfft_ragged_get_report(tfft_ragged r, tfft_counts *counts, tfft_record *recs, int64_t cap) {
    if (!r || cap < 0 || (cap > 0 && !recs)) return TFFT_E_INVALID;
    if (!r->executed) return TFFT_E_STATE;
    Guard guard(r->device);
    if (hipStreamSynchronize(r->last_stream) != hipSuccess) return TFFT_E_HIP;
    tfft_counts total;
    std::memset(&total, 0, sizeof(total));
    int status = TFFT_OK;
    std::vector<tfft_record> all;
    if (r->persistent) {
        // one report for every class: records carry their task (class, pass)
        DevReport h;
        int32_t err = 0;
        if (hipMemcpy(&h, r->d_rep, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&err, r->d_err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
            return TFFT_E_HIP;
        if (err) return TFFT_E_HIP;  // a dependency wait gave up: the outputs are not to be trusted
        const int64_t nrec = std::min<int64_t>((int64_t)h.n_flag, r->rec_cap);
        std::vector<DevRecord> dr((size_t)nrec);
        if (nrec > 0 &&
            hipMemcpy(dr.data(), r->d_recs, sizeof(DevRecord) * (size_t)nrec, hipMemcpyDeviceToHost) != hipSuccess)
            return TFFT_E_HIP;
        if (r->last_mode != TFFT_FT_OFF)
            for (auto &C : r->classes)
                for (int i = 0; i < C.plan->passes; ++i) total.groups_checked += C.plan->pass[i].n_groups;
        total.detected = (int64_t)h.n_flag;
        total.corrected = (int64_t)h.corrected;
        total.uncorrectable = (int64_t)h.uncorrectable;
        total.benign = (int64_t)h.benign;
        total.n_records = nrec;
        total.dropped = (int64_t)h.n_flag - nrec;
        for (const DevRecord &d : dr) {
            if (d.task < 0 || d.task >= (int)r->task_class.size()) continue;
            const auto &C = r->classes[(size_t)r->task_class[(size_t)d.task]];
            tfft_record x = host_record(C.plan, d);
            x.signal = C.members[(size_t)x.signal];
            all.push_back(x);
        }
        if (h.uncorrectable > 0 || (r->last_mode == TFFT_FT_CORRECT && total.dropped > 0)) status = TFFT_UNCORRECTABLE;
    }
    for (auto &C : r->classes) {
        if (r->persistent) break;
        tfft_counts c;
        int rc = tfft_get_report(C.plan, &c, nullptr, 0);
        if (rc < 0) return rc;
        std::vector<tfft_record> v((size_t)c.n_records);
        rc = tfft_get_report(C.plan, &c, v.data(), c.n_records);
        if (rc < 0) return rc;
        if (rc == TFFT_UNCORRECTABLE) status = TFFT_UNCORRECTABLE;
        total.groups_checked += c.groups_checked;
        total.detected += c.detected;
        total.corrected += c.corrected;
        total.uncorrectable += c.uncorrectable;
        total.benign += c.benign;
        total.n_records += c.n_records;
        total.dropped += c.dropped;
        for (auto &x : v) {
            x.signal = C.members[(size_t)x.signal];
            all.push_back(x);
        }
    }
    std::sort(all.begin(), all.end(), [](const tfft_record &x, const tfft_record &y) {
        if (x.signal != y.signal) return x.signal < y.signal;
        if (x.pass != y.pass) return x.pass < y.pass;
        if (x.group != y.group) return x.group < y.group;
        return x.sub < y.sub;
    });
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)all.size()); ++i) recs[i] = all[(size_t)i];
    if (counts) *counts = total;
    return status;
}

int tfft_ragged_set_faults(tfft_ragged r, const tfft_fault *specs, int64_t n) {
    if (!r || n < 0 || (n > 0 && !specs)) return TFFT_E_INVALID;
    std::vector<std::vector<tfft_fault>> per(r->classes.size());
    for (int64_t k = 0; k < n; ++k) {
        if (specs[k].signal < 0 || specs[k].signal >= r->count) return TFFT_E_INVALID;
        tfft_fault f = specs[k];
        const size_t c = (size_t)r->class_of[(size_t)f.signal];
        f.signal = r->local_of[(size_t)f.signal];
        per[c].push_back(f);
    }
    drop_graph(r);
    r->tasks_valid = 0;  // the tasks point at the fault tables
    if (r->persistent && r->executed) {
        // the fault tables are replaced: wait for the last execution that reads them
        Guard guard(r->device);
        if (hipStreamSynchronize(r->last_stream) != hipSuccess) return TFFT_E_HIP;
    }
    for (size_t c = 0; c < r->classes.size(); ++c) {
        const int rc = tfft_set_faults(r->classes[c].plan, per[c].data(), (int64_t)per[c].size());
        if (rc != TFFT_OK) return rc;
    }
    r->class_faults = std::move(per);
    return TFFT_OK;
}

int tfft_ragged_tune(tfft_ragged r, const void *d_in, void *d_out, void *hip_stream, int reps) {
    if (!r || !d_in || !d_out || reps < 1) return TFFT_E_INVALID;
    Guard guard(r->device);
    hipStream_t st = (hipStream_t)hip_stream;
    if (r->persistent) return persist_tune(r, d_in, d_out, st, reps);
    drop_graph(r);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TFFT_E_HIP;
    int status = TFFT_OK;
    for (size_t ci = 0; ci < r->classes.size() && status == TFFT_OK; ++ci) {
        auto &C = r->classes[ci];
        const int k = ilog2_64(C.n);
        // candidates: pass count, checksum group size, workgroups per launch
        std::vector<tfft_options> cand;
        for (int ps = 1; ps <= 3; ++ps) {
            if ((ps == 1 && k > TFFT_ONE_PASS_MAX_LOG2) || (ps == 2 && (k < 8 || k > 20)) || (ps == 3 && k < 12)) continue;
            for (int grp : {0, 16, 64})
                for (int gs : {-1, 0, 1}) {
                    tfft_options o = r->opt;
                    o.passes = ps;
                    o.group = grp;
                    o.grid_scale = gs;
                    cand.push_back(o);
                }
        }
        float best = 1e30f;
        tfft_options best_opt = r->opt;
        for (const auto &o : cand) {
            if (build_class(r, ci, o) != TFFT_OK) continue;  // unsupported candidate
            float ms = 0.f;
            bool ok = true;
            for (int t = 0; t <= reps && ok; ++t) {  // first run warms up
                if (t == 1 && hipEventRecord(e0, st) != hipSuccess) ok = false;
                if (exec(C.plan, d_in, d_out, TFFT_FT_CORRECT, st, false) != TFFT_OK) ok = false;
            }
            if (ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ok && ms < best) {
                best = ms;
                best_opt = o;
            }
        }
        status = build_class(r, ci, best_opt);
        // the new plan gets the faults installed on the old one
        if (status == TFFT_OK && ci < r->class_faults.size() && !r->class_faults[ci].empty())
            status = tfft_set_faults(C.plan, r->class_faults[ci].data(), (int64_t)r->class_faults[ci].size());
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

int tfft_ragged_info(tfft_ragged r, int64_t *classes, int64_t *lengths, int64_t *counts, tfft_plan_desc *descs,
                     int64_t cap) {
    if (!r || cap < 0) return TFFT_E_INVALID;
    if (classes) *classes = (int64_t)r->classes.size();
    for (int64_t c = 0; c < std::min<int64_t>(cap, (int64_t)r->classes.size()); ++c) {
        if (lengths) lengths[c] = r->classes[(size_t)c].n;
        if (counts) counts[c] = (int64_t)r->classes[(size_t)c].members.size();
        if (descs) tfft_plan_info(r->classes[(size_t)c].plan, &descs[c]);
    }
    return TFFT_OK;
}

int tfft_plan_describe(int64_t n, int64_t batch, int dtype, const tfft_options *opt, tfft_plan_desc *info) {
    if (!info) return TFFT_E_INVALID;
    tfft_plan_s *p = new (std::nothrow) tfft_plan_s();
    if (!p) return TFFT_E_NOMEM;
    int rc = shape_plan(p, n, batch, dtype, opt, false);
    if (rc == TFFT_OK) rc = tfft_plan_info(p, info);
    delete p;  // owns no device memory
    return rc;
}

int tfft_host_root(int64_t t, int64_t n, double *out) {
    if (!out || n < 1) return TFFT_E_INVALID;
    const cd w = unit_root(t, n);
    out[0] = w.real();
    out[1] = w.imag();
    return TFFT_OK;
}

int tfft_host_checksum_vector(int64_t m, int inverse, double scale, double *out) {
    if (!out || m < 2 || m > (int64_t(1) << 24) || (m & (m - 1)) != 0 || !std::isfinite(scale)) return TFFT_E_INVALID;
    const std::vector<double> c = checksum_vec((int)m, inverse != 0, scale);
    std::memcpy(out, c.data(), sizeof(double) * c.size());
    return TFFT_OK;
}

int tfft_plan_info(tfft_plan p, tfft_plan_desc *info) {
    if (!p || !info) return TFFT_E_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->n = p->n;
    info->batch = p->batch;
    info->dtype = p->dtype;
    info->passes = p->passes;
    for (int i = 0; i < p->passes; ++i) {
        const PassPlan &P = p->pass[i];
        info->pass_len[i] = P.M;
        info->group[i] = P.G;
        info->elems_per_thread[i] = P.E;
        info->tile_signals[i] = P.C;
        info->stages[i] = P.stages;
        for (int s = 0; s < P.stages && s < 8; ++s) info->radices[i][s] = stage_radix(P.M, P.E, s);
        info->groups[i] = P.n_groups;
    }
    info->workspace_bytes = p->work_bytes;
    info->kappa = p->kappa;
    return TFFT_OK;
}

}  // extern "C"
