// Host driver of block GCRO-DR (Algorithm 1) on one MI355X and the C ABI of
// libbgcr.so.  Every n-sized operation runs in the HIP kernels of kernels.hip;
// the host keeps only the small FP64 problems of each cycle (least-squares
// back substitution, harmonic Ritz eigenproblem, QR of G P) whose size is
// independent of n.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "bgcr.h"
#include "bgcr_internal.h"
#include "dense.h"

using namespace bgcr;
using dense::cd;
using dense::Mat;

struct bgcr_sequence {
    virtual ~bgcr_sequence() {}
    virtual int solve(const bgcr_csr* A, const void* B, int64_t ldb, void* X, int64_t ldx, double tol,
                      bgcr_stats* st) = 0;
    virtual int get_recycle(void* U, void* C, int64_t ld) const = 0;
    virtual int set_recycle(const void* U, int64_t ld, int k_in) = 0;
    virtual int recycle_dim() const = 0;
    virtual void set_profiling(int on) = 0;
    virtual void get_profile(double* ms, double* bytes, int64_t* launches, int nclass) const = 0;
    virtual void set_cycle_limit(int cycles) = 0;  // restart cycles per solve from now on
    std::vector<int> log_steps;
    std::vector<double> log_res;
};

namespace {

inline cd to_cd(double v) { return cd(v, 0.0); }
inline cd to_cd(zd v) { return cd(v.x, v.y); }
template <class A> A from_cd(cd v);
template <> double from_cd<double>(cd v) { return v.real(); }
template <> zd from_cd<zd>(cd v) { return {v.real(), v.imag()}; }

struct Fail {
    int code;
};
#define HIPCHK(...)                                      \
    do {                                                 \
        hipError_t e_ = (__VA_ARGS__);                   \
        if (e_ != hipSuccess) throw Fail{BGCR_ERR_HIP};  \
    } while (0)

// block size of the Krylov basis: p, or the enlarged size for p = 1
int block_of(const bgcr_params* prm) { return prm->block_size > 0 ? prm->block_size : prm->p; }

bool valid_params(const bgcr_params* prm, int64_t n) {
    if (!prm || n <= 0) return false;
    const int pu = prm->p;
    if (!(pu == 1 || pu == 2 || pu == 4 || pu == 8 || pu == 16)) return false;
    const int bs = prm->block_size;
    if (bs != 0 && bs != pu && !(pu == 1 && (bs == 2 || bs == 4 || bs == 8 || bs == 16))) return false;
    const int p = block_of(prm);
    if (prm->m < 1 || prm->m > 64 || prm->k < 0 || prm->k > 128) return false;
    if (prm->dtype != BGCR_F64 && prm->dtype != BGCR_C128) return false;
    if (prm->precision != BGCR_PLAIN_FP64 && prm->precision != BGCR_MIXED_FP32 &&
        prm->precision != BGCR_MIXED_FP32_BF16)
        return false;
    if (prm->dtype == BGCR_C128 && prm->precision != BGCR_PLAIN_FP64) return false;
    // BF16 basis storage runs on the matrix-core sweeps only (P = 8 or 16)
    if (prm->precision == BGCR_MIXED_FP32_BF16 && !(p == 8 || p == 16)) return false;
    if (prm->max_cycles < 1) return false;
    // the hybrid needs an enlarged block and a basis type the L = 1 basis has
    if (prm->enlarge_cycles < 0) return false;
    if (prm->ritz_vectors != 0 && prm->ritz_vectors != 1) return false;
    if (prm->precond != BGCR_PRECOND_NONE && prm->precond != BGCR_PRECOND_ILU0) return false;
    // ILU(0): plain FP64 (real or complex), no enlarged block, no hybrid
    if (prm->precond == BGCR_PRECOND_ILU0 &&
        (prm->precision != BGCR_PLAIN_FP64 || p != pu || prm->enlarge_cycles != 0))
        return false;
    if (prm->enlarge_cycles > 0 && (p == pu || prm->precision == BGCR_MIXED_FP32_BF16)) return false;
    const int KB = (prm->k + (prm->dtype == BGCR_F64 ? 1 : 0) + p - 1) / p;
    // the refresh combines [U, C, V_1 .. V_{m+1}] in one launch
    if (2 * KB + prm->m + 1 > MAXB) return false;
    if ((KB + prm->m) * p * p > MAXI * NT) return false;
    return true;
}

struct Sizes {
    int P, m, k, KB, KP;
    size_t s, sw, sa;  // bytes of a basis scalar, of a work-block scalar (W, R), of an FP64 scalar
    size_t basis, blk, recyc, small_, part, total_fixed;
    size_t nout;   // outputs per workgroup of the reduction partials
};

// outputs per workgroup of the largest reduction: an Arnoldi sweep (q x P)
// or a recycle dot launch (up to 32 W columns, at most KB blocks, against q)
size_t part_outputs(int P, int KB, int qmax, bool cplx) {
    const size_t wg = (size_t)std::max(1, std::min(KB, std::max(1, 32 / P)));
    // the second pass of a block step writes its dots and the new block's Gram
    const size_t o = std::max({(size_t)qmax * P + (size_t)P * P, (size_t)KB * P * P, wg * qmax * P});
    // complex sweeps on matrix cores write the real 2q x 2P products (twice
    // the complex entries), the second pass followed by the real Gram
    return cplx ? std::max(o, 2 * ((size_t)qmax * P + (size_t)P * P)) : o;
}

Sizes sizes_of(const bgcr_params* prm, int64_t n) {
    Sizes z;
    z.P = block_of(prm);
    z.m = prm->m;
    z.k = prm->k;
    const bool cplx = prm->dtype == BGCR_C128;
    z.KB = z.k > 0 ? (z.k + (cplx ? 0 : 1) + z.P - 1) / z.P : 0;
    z.KP = z.KB * z.P;
    z.sa = cplx ? 16 : 8;
    z.sw = cplx ? 16 : (prm->precision == BGCR_PLAIN_FP64 ? 8 : 4);
    z.s = prm->precision == BGCR_MIXED_FP32_BF16 ? 2 : z.sw;
    z.blk = (size_t)n * z.P * z.s;
    z.basis = (size_t)(z.m + 1) * z.blk;  // V_1 .. V_{m+1}
    z.recyc = 4 * (size_t)z.KB * z.blk;
    const int qmax = (2 * z.KB + z.m + 1) * z.P;
    z.nout = part_outputs(z.P, z.KB, qmax, cplx);
    z.part = (size_t)NWG_MAX * z.nout * z.sa;
    const size_t mp = (size_t)z.m * z.P, m1p = (size_t)(z.m + 1) * z.P;
    z.small_ = z.sa * (2 * (size_t)qmax * z.P + (size_t)z.P * z.P + 2 * m1p * mp + (size_t)z.KP * mp + (size_t)z.m * 4 * z.P * z.P +
                       m1p * z.P + (size_t)(z.m + 1) * z.P * z.P + 2 * (size_t)z.P * z.P +
                       (size_t)(2 * z.KB + z.m + 1) * z.P * (2 * std::max(z.KP, z.P) + 2 * z.P)) +
               sizeof(double) * ((size_t)z.m + (size_t)NWG_MAX * 2 * z.P) + sizeof(Ctl) +
               (cplx ? sizeof(double) * 4 * (size_t)(z.KB + z.m + 1) * z.P * z.P : 0);
    const bool enlarged = z.P > prm->p;
    z.total_fixed = z.basis + 3 * (size_t)n * z.P * z.sw /* W2, Wb, R */ +
                    (size_t)n * z.P * z.sa * (enlarged ? 2 : 1) /* X (and B padded) */ + z.recyc + z.part + z.small_;
    // ILU(0): the two blocks of M^{-1}, diagonal positions, the analysed row
    // pointers, a flag and two ticket counters (the nnz-sized arrays and the
    // level orders are counted by bgcr_footprint_bytes)
    if (prm->precond == BGCR_PRECOND_ILU0)
        z.total_fixed += 2 * (size_t)n * z.P * z.sw + sizeof(int) * (2 * (size_t)n + 4);
    return z;
}

}  // namespace

// T: storage and arithmetic type of the work blocks (W, R, the start block)
// and of the matrix copy of the cycles; TB: storage type of the basis blocks
// (V, U, C), T itself or BF16 (FP32 form with BF16 basis storage).
template <class T, class TB = T>
struct Seq final : bgcr_sequence {
    using A = acc_t<T>;  // FP64 real or complex128: coefficients, solution, matrix for the residual
    using L = Launch<T>;
    static constexpr bool half = !std::is_same<T, TB>::value;  // basis stored in BF16

    bgcr_params prm;
    int64_t n;
    int P, m, k, KB, KP, nwg;
    int pu = 0;  // right-hand sides of the caller (P > pu: enlarged block, pu = 1)
    int nwg_mx = 0;      // workgroups of the matrix-core sweeps (64-row tiles)
    bool use_mx = false; // Arnoldi sweeps on matrix cores
    // Sweep directions alternate, so that every sweep of a block step starts
    // on the rows the one before it read last, which the chip's memory-side
    // cache still holds (third sweep 295 -> 277 us, second 231 -> 226 us at
    // 128^3, p = 8).  Step 1: SpMM and third sweep forwards, first-pass dots
    // backwards; later steps, after the fused SpMM + dots (forwards): second
    // sweep backwards, third forwards.
    static constexpr bool alt_dir = true;
    // sweeps 1a and 1b fused into one pass (real FP64 on matrix cores)
    bool fuse_dots = false;
    bool mx_dot = false; // dot sweeps on matrix cores (also narrow real blocks, P < 8)
    bool mx_upd = false; // update sweeps on matrix cores (also P = 4, without the PIP step order)
    bool cx_mx = false;  // complex block-CGS sweeps on the FP64 matrix cores (P = 8 or 16)
    bool pip_order = false;  // block steps in the PIP order (V_{j+1} stored normalised by the third sweep)
    double* Sr = nullptr;  // real form of a complex coefficient matrix (cx_mx, P = 8)
    bool mixed, cplx;
    hipStream_t st;
    Sizes sz;

    TB* Vb = nullptr;
    T *W2 = nullptr, *Wb = nullptr, *R = nullptr;
    TB* Ub[2] = {nullptr, nullptr};
    TB* Cb[2] = {nullptr, nullptr};
    A* X = nullptr;
    A* Bpad = nullptr;  // B padded to P columns (enlarged block)
    float* av32 = nullptr;
    size_t av32_cap = 0;
    A* dots = nullptr;
    size_t dots_cap = 0;
    unsigned char* hr = nullptr;  // host-read region (see the constructor)
    size_t off_H = 0, off_Rh = 0, off_g = 0, off_Ri = 0, off_F = 0, off_dots = 0, hr_bytes = 0;
    size_t part_cap = 0;  // elements of `part`
    A *part = nullptr, *S1 = nullptr, *Sf = nullptr, *H = nullptr, *F = nullptr, *Rh = nullptr, *QH = nullptr,
      *g = nullptr, *RinvAll = nullptr, *Z1 = nullptr, *Z1i = nullptr, *coef = nullptr;
    size_t coef_cap = 0;
    double *rho = nullptr, *dpart = nullptr;
    Ctl* ctl = nullptr;
    unsigned char* hbuf = nullptr;
    size_t hcap = 0, hoff = 0;
    double* rbuf = nullptr;  // pinned: residual partials copied back while the host works
    hipEvent_t ev_res = nullptr;  // recorded after the copy of the residual partials
    A* dbuf = nullptr;               // pinned: the refresh dots, copied back after the steps' results
    hipEvent_t ev_cyc = nullptr, ev_dots = nullptr;  // after the copies of the steps' results, of the dots
    int cur = 0, keff = 0;
    // per-solve counters
    int n_spmm = 0, n_steps = 0, n_cycles = 0, n_refine = 0;
    double alg_bytes = 0.0;
    int n_deflated = 0;  // rank-deficient blocks handled: start blocks rebuilt, cycles ended at a breakdown

    // ILU(0) right preconditioning: level schedule of the analysed pattern,
    // the factors of the current system, and the two blocks of M^{-1} (Yb
    // holds L^{-1} in, Zb the result)
    bool pc = false;
    int *d_rp = nullptr, *d_ci = nullptr, *d_diag = nullptr, *d_ordL = nullptr, *d_ordU = nullptr,
        *d_flag = nullptr;
    unsigned* d_tick = nullptr;   // ticket counters of the L and U solves
    bool ilu_used = false;        // this solve factored its system
    int64_t pat_nnz = -1;         // nnz of the analysed pattern (-1: none yet)
    size_t ci_cap = 0, lu_cap = 0, ordL_cap = 0, ordU_cap = 0;
    std::vector<int> lvlL, lvlU;  // level pointers into the padded L and U row orders
    A* lu = nullptr;
    T *Zb = nullptr, *Yb = nullptr;

    std::vector<void*> allocs;

    // opt-in per-kernel-class timing with HIP events on this sequence's stream
    struct Pend {
        int cls, step;
        double bytes;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<hipEvent_t> evfree;
    std::vector<Pend> pend;
    double pms[BGCR_K_NCLASS] = {}, pby[BGCR_K_NCLASS] = {};
    long long pcnt[BGCR_K_NCLASS] = {};
    int cur_step = 0;  // block step of the launches being enqueued (0: not a step kernel)

    hipEvent_t ev_get() {
        if (evfree.empty()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = evfree.back();
        evfree.pop_back();
        return e;
    }
    template <class FN>
    void run(int cls, double bytes, FN&& launch) {
        if (!prof) {
            HIPCHK(launch());
            return;
        }
        if (pend.size() > 16384) prof_resolve(1 << 30);
        hipEvent_t a = ev_get(), b = ev_get();
        HIPCHK(hipEventRecord(a, st));
        HIPCHK(launch());
        HIPCHK(hipEventRecord(b, st));
        pend.push_back({cls, cur_step, bytes, a, b});
    }
    // accumulate finished launches; step kernels beyond `meff` were skipped on
    // the device (early exit of the cycle) and are not counted
    void prof_resolve(int meff) {
        if (pend.empty()) return;
        HIPCHK(hipStreamSynchronize(st));
        for (const Pend& q : pend) {
            if (q.step <= meff) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, q.a, q.b));
                pms[q.cls] += ms;
                pby[q.cls] += q.bytes;
                pcnt[q.cls] += 1;
            }
            evfree.push_back(q.a);
            evfree.push_back(q.b);
        }
        pend.clear();
    }
    // wall-clock time of a host-side phase, recorded while profiling
    struct HostPhase {
        Seq* s;
        int cls;
        std::chrono::steady_clock::time_point t0;
        HostPhase(Seq* s_, int c) : s(s_), cls(c), t0(std::chrono::steady_clock::now()) {}
        ~HostPhase() {
            if (!s->prof) return;
            s->pms[cls] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            s->pcnt[cls] += 1;
        }
    };
    void set_profiling(int on) override {
        prof_resolve(1 << 30);
        prof = on != 0;
        for (int c = 0; c < BGCR_K_NCLASS; ++c) {
            pms[c] = pby[c] = 0.0;
            pcnt[c] = 0;
        }
    }

    Seq(const bgcr_params* p_, int64_t n_, hipStream_t s_) : prm(*p_), n(n_), st(s_) {
        P = block_of(&prm);
        pu = prm.p;
        pc = prm.precond == BGCR_PRECOND_ILU0;
        m = prm.m;
        k = prm.k;
        cplx = prm.dtype == BGCR_C128;
        mixed = prm.precision != BGCR_PLAIN_FP64;
        sz = sizes_of(&prm, n);
        KB = sz.KB;
        KP = sz.KP;
        nwg = nwg_for(n, P);
        nwg_mx = mfma_nwg(n);
        const char* e = std::getenv("BGCR_NO_MFMA");
        const bool off = e && e[0] == '1';
        use_mx = !off && !std::is_same<T, zd>::value && (P == 8 || P == 16) &&
                 (KB + m) * P <= (P == 16 && sizeof(T) == 8 ? 224 : 256);
        const bool realb = !std::is_same<T, zd>::value && !half;
        mx_dot = use_mx || (realb && !off && P < 8);
        mx_upd = use_mx || (realb && !off && P == 4 && (KB + m) * P <= 256);
        fuse_dots = use_mx && std::is_same<T, double>::value && !half;
        cx_mx = !off && std::is_same<T, zd>::value && (P == 8 || P == 16) && KB + m <= cx_mfma_max_blocks(P, false);
        pip_order = use_mx || (cx_mx && KB + m <= cx_mfma_max_blocks(P, true));
        // BF16 basis blocks have matrix-core kernels only; every basis
        // combination has to fit one launch (at most 64 output columns)
        if (half && (!use_mx || 2 * KP > 64 ||
                     ((size_t)(2 * KB + m + 1) * P * 16 * ((2 * KP + 15) / 16) + 4 * 16 * 64) * sizeof(double) >
                         (size_t)160 * 1024))
            throw Fail{BGCR_ERR_INVALID};
    }

    ~Seq() override {
        (void)hipStreamSynchronize(st);
        for (const Pend& q : pend) {
            (void)hipEventDestroy(q.a);
            (void)hipEventDestroy(q.b);
        }
        for (hipEvent_t e : evfree) (void)hipEventDestroy(e);
        if (ev_res) (void)hipEventDestroy(ev_res);
        if (ev_cyc) (void)hipEventDestroy(ev_cyc);
        if (ev_dots) (void)hipEventDestroy(ev_dots);
        if (dbuf) (void)hipHostFree(dbuf);
        for (void* p : allocs) (void)hipFree(p);
        if (hbuf) (void)hipHostFree(hbuf);
        if (rbuf) (void)hipHostFree(rbuf);
    }

    template <class U_>
    U_* dalloc(size_t count) {
        if (count == 0) return nullptr;
        void* p = nullptr;
        if (hipMalloc(&p, count * sizeof(U_)) != hipSuccess) throw Fail{BGCR_ERR_NOMEM};
        allocs.push_back(p);
        // every workspace starts defined (zero)
        HIPCHK(hipMemsetAsync(p, 0, count * sizeof(U_), st));
        return (U_*)p;
    }

    void allocate() {
        const size_t blk = (size_t)n * P;
        Vb = dalloc<TB>((size_t)(m + 1) * blk);
        W2 = dalloc<T>(blk);
        Wb = dalloc<T>(blk);
        R = dalloc<T>(blk);
        X = dalloc<A>(blk);
        if (P > pu) Bpad = dalloc<A>(blk);
        for (int i = 0; i < 2; ++i) {
            Ub[i] = dalloc<TB>((size_t)KB * blk);
            Cb[i] = dalloc<TB>((size_t)KB * blk);
        }
        const int qmax = (2 * KB + m + 1) * P;
        part_cap = (size_t)NWG_MAX * sz.nout;
        part = dalloc<A>(part_cap);
        S1 = dalloc<A>((size_t)qmax * P);
        dots_cap = (size_t)qmax * P * std::max(KB, 1);
        Sf = dalloc<A>((size_t)qmax * P + (size_t)P * P);  // [S1 + S2 | W'^H W']
        if (cx_mx) Sr = dalloc<double>(4 * (size_t)(KB + m + 1) * P * P);  // S_r, then R^{-1}_r
        const size_t mp = (size_t)m * P, m1p = (size_t)(m + 1) * P;
        // everything the host reads at the end of a cycle, contiguous so that
        // one copy brings it over: control block, H and its triangular factor,
        // g, R^{-1} of every step, F and the refresh dot products
        {
            auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
            off_H = al(sizeof(Ctl));
            off_Rh = off_H + al(m1p * mp * sizeof(A));
            off_g = off_Rh + al(m1p * mp * sizeof(A));
            off_Ri = off_g + al(m1p * P * sizeof(A));
            off_F = off_Ri + al((size_t)(m + 1) * P * P * sizeof(A));
            off_dots = off_F + al(std::max<size_t>(1, (size_t)KP * mp) * sizeof(A));
            hr_bytes = off_dots + al(dots_cap * sizeof(A));
            hr = dalloc<unsigned char>(hr_bytes);
            ctl = (Ctl*)hr;
            H = (A*)(hr + off_H);
            Rh = (A*)(hr + off_Rh);
            g = (A*)(hr + off_g);
            RinvAll = (A*)(hr + off_Ri);
            F = (A*)(hr + off_F);
            dots = (A*)(hr + off_dots);
        }
        QH = dalloc<A>((size_t)m * 4 * P * P);
        Z1 = dalloc<A>((size_t)P * P);
        Z1i = dalloc<A>((size_t)P * P);
        coef_cap = (size_t)(2 * KB + m + 1) * P * (2 * std::max(KP, P) + 2 * P);
        coef = dalloc<A>(coef_cap);
        rho = dalloc<double>(m);
        dpart = dalloc<double>((size_t)NWG_MAX * 2 * P);
        if (pc) {
            Zb = dalloc<T>(blk);
            Yb = dalloc<T>(blk);
            d_rp = dalloc<int>((size_t)n + 1);
            d_diag = dalloc<int>((size_t)n);
            d_flag = dalloc<int>(1);
            d_tick = dalloc<unsigned>(2);
        }
        hcap = std::max({(size_t)4 << 20, 2 * coef_cap * sizeof(A) + (64 << 10), hr_bytes + (64 << 10)});
        if (hipHostMalloc((void**)&hbuf, hcap, hipHostMallocDefault) != hipSuccess) throw Fail{BGCR_ERR_NOMEM};
        if (hipHostMalloc((void**)&dbuf, std::max<size_t>(1, dots_cap) * sizeof(A), hipHostMallocDefault) != hipSuccess)
            throw Fail{BGCR_ERR_NOMEM};
        HIPCHK(hipEventCreateWithFlags(&ev_cyc, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev_dots, hipEventDisableTiming));
        if (hipHostMalloc((void**)&rbuf, (size_t)NWG_MAX * 2 * P * sizeof(double), hipHostMallocDefault) != hipSuccess)
            throw Fail{BGCR_ERR_NOMEM};
        HIPCHK(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
        HIPCHK(hipMemsetAsync(Ub[0], 0, (size_t)KB * blk * sizeof(TB), st));
        HIPCHK(hipMemsetAsync(Ub[1], 0, (size_t)KB * blk * sizeof(TB), st));
        HIPCHK(hipMemsetAsync(Cb[0], 0, (size_t)KB * blk * sizeof(TB), st));
        HIPCHK(hipMemsetAsync(Cb[1], 0, (size_t)KB * blk * sizeof(TB), st));
        HIPCHK(hipStreamSynchronize(st));
    }

    TB* vblk(int j) { return Vb + (size_t)j * n * P; }
    TB* ublk(int buf, int b) { return Ub[buf] + (size_t)b * n * P; }
    TB* cblk(int buf, int b) { return Cb[buf] + (size_t)b * n * P; }

    // ---- host <-> device staging through pinned memory --------------------
    void sync() {
        HIPCHK(hipStreamSynchronize(st));
        hoff = 0;
        if (prof && cur_step == 0) prof_resolve(1 << 30);
    }
    void d2h(void* dst, const void* src, size_t bytes) {
        if (bytes == 0) return;
        sync();
        size_t done = 0;
        while (done < bytes) {
            const size_t c = std::min(bytes - done, hcap);
            HIPCHK(hipMemcpyAsync(hbuf, (const char*)src + done, c, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::memcpy((char*)dst + done, hbuf, c);
            done += c;
        }
    }
    // several device -> host copies with a single synchronisation
    struct Copy {
        void* dst;
        const void* src;
        size_t bytes;
    };
    void d2h_many(const std::vector<Copy>& cps) {
        size_t tot = 0;
        for (const Copy& c : cps) tot += (c.bytes + 255) & ~(size_t)255;
        if (tot > hcap) {
            for (const Copy& c : cps) d2h(c.dst, c.src, c.bytes);
            return;
        }
        sync();
        size_t off = 0;
        for (const Copy& c : cps) {
            if (c.bytes) HIPCHK(hipMemcpyAsync(hbuf + off, c.src, c.bytes, hipMemcpyDeviceToHost, st));
            off += (c.bytes + 255) & ~(size_t)255;
        }
        HIPCHK(hipStreamSynchronize(st));
        off = 0;
        for (const Copy& c : cps) {
            if (c.bytes) std::memcpy(c.dst, hbuf + off, c.bytes);
            off += (c.bytes + 255) & ~(size_t)255;
        }
    }

    void h2d(void* dst, const void* src, size_t bytes) {
        if (bytes == 0) return;
        if (bytes > hcap) throw Fail{BGCR_ERR_INVALID};
        const size_t al = (bytes + 255) & ~(size_t)255;
        if (hoff + al > hcap) sync();
        std::memcpy(hbuf + hoff, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, hbuf + hoff, bytes, hipMemcpyHostToDevice, st));
        hoff += al;
    }

    static BlockPtrs bp(const std::vector<const void*>& v) {
        BlockPtrs b;
        std::memset(&b, 0, sizeof(b));
        if (v.size() > (size_t)MAXB) throw Fail{BGCR_ERR_INVALID};
        for (size_t i = 0; i < v.size(); ++i) b.p[i] = v[i];
        return b;
    }

    // Upload a coefficient matrix K ((nin P) x (nout P)) for k_combine.
    const A* upload_coef(const Mat& K, int nin, int nout, A* dst) {
        const size_t cnt = (size_t)nin * nout * P * P;
        std::vector<A> h(cnt);
        for (int i = 0; i < nin; ++i)
            for (int o = 0; o < nout; ++o)
                for (int a = 0; a < P; ++a)
                    for (int b = 0; b < P; ++b) {
                        const int rr = i * P + a, cc = o * P + b;
                        const cd v = (rr < K.r && cc < K.c) ? K(rr, cc) : cd(0.0, 0.0);
                        h[(((size_t)i * P + a) * nout + o) * P + b] = from_cd<A>(v);
                    }
        h2d(dst, h.data(), cnt * sizeof(A));
        return dst;
    }

    // inputs are basis blocks (TB), or work blocks when TB is T
    template <class TO>
    void combine(const std::vector<const void*>& in, const std::vector<void*>& out, const Mat& K, int accumulate) {
        const int nin = (int)in.size(), nout = (int)out.size();
        if ((size_t)nin * nout * P * P > coef_cap) throw Fail{BGCR_ERR_INVALID};
        std::vector<const void*> outc(out.begin(), out.end());
        const A* cf = upload_coef(K, nin, nout, coef);
        const double by = (double)n * P * ((double)sizeof(TB) * nin + (double)sizeof(TO) * (nout + accumulate));
        run(BGCR_K_COMBINE, by, [&] {
            if constexpr (!std::is_same<T, zd>::value) {
                // matrix cores: the Arnoldi configurations, and four-column FP64 blocks
                if (use_mx || (P == 4 && std::is_same<TB, double>::value)) {
                    const hipError_t e =
                        mfma_combine<TB, TO>(st, P, n, bp(in), nin, bp(outc), nout, cf, accumulate, nwg_mx);
                    if (e != hipErrorNotSupported) return e;
                }
            } else {
                if (cx_mx) {
                    const hipError_t e = cx_combine(st, P, n, bp(in), nin, bp(outc), nout, cf, accumulate, nwg_mx);
                    if (e != hipErrorNotSupported) return e;
                }
            }
            if constexpr (half) {
                return hipErrorNotSupported;
            } else {
                return L::template combine<TO>(st, P, n, bp(in), nin, bp(outc), nout, cf, accumulate);
            }
        });
    }

    // Q^H W for a list of W blocks: returns Mat (nq P) x (nw P).  Every piece
    // is reduced into its own slice of `dots`; one copy to the host at the end.
    // Q^H W for a list of W blocks, as (nq P) x (nw P): enqueued pieces reduced
    // into consecutive slices of `dots`, assembled on the host by dot_collect
    struct DotJob {
        struct Piece {
            int w0, wn, q0, qn;
            size_t off;
        };
        std::vector<Piece> pieces;
        size_t total = 0;  // elements of `dots` written
        int nq = 0, nw = 0;
        bool valid = false;
    };

    // Q: basis blocks (TB); W: blocks of type TW (TB or T)
    template <class TW>
    DotJob dot_enqueue(const std::vector<const void*>& Q, const std::vector<const TW*>& W) {
        DotJob job;
        job.nq = (int)Q.size();
        job.nw = (int)W.size();
        const int nq = job.nq, nw = job.nw;
        // per launch: wg W blocks (32 columns on matrix cores, so that one pass
        // over a Q chunk serves them all) against a chunk of Q blocks.  The
        // matrix-core dot also serves narrow real blocks (P < 8), where a
        // 16-column chunk spans 16 / P blocks (at most MAXB per launch).
        const bool mxd = mx_dot;
        const bool cxd = cx_mx;  // complex blocks on the FP64 matrix cores, one W block per launch
        const int wg = mxd ? std::max(1, 32 / P) : 1;
        const int nr = (mxd || cxd) ? nwg_mx : nwg;
        if ((size_t)nq * P * P * nw > dots_cap) throw Fail{BGCR_ERR_INVALID};
        size_t off = 0;
        for (int w0 = 0; w0 < nw; w0 += wg) {
            const int wn = std::min(wg, nw - w0);
            const int ng = (wn * P + 15) / 16;
            const int chunk = mxd   ? std::max(1, std::min((ng == 2 ? 9 : 16) * 16 / P, MAXB))
                              : cxd ? cx_mfma_max_blocks(P, false)
                                    : std::max(1, (MAXI * NT) / (P * P));
            for (int q0 = 0; q0 < nq; q0 += chunk) {
                const int qn = std::min(chunk, nq - q0);
                const int nout = wn * qn * P * P;
                // (the real partials of complex blocks take twice the entries)
                if ((size_t)nr * nout * (cxd ? 2 : 1) > part_cap) throw Fail{BGCR_ERR_INVALID};
                std::vector<const void*> sub(Q.begin() + q0, Q.begin() + q0 + qn);
                std::vector<const void*> ws(W.begin() + w0, W.begin() + w0 + wn);
                run(BGCR_K_TSDOT, (double)n * P * ((double)sizeof(TW) * wn + (double)sizeof(TB) * qn), [&] {
                    if constexpr (!std::is_same<T, zd>::value) {
                        if (mxd) return mfma_dot<T, TW, TB>(st, P, n, bp(ws), wn, bp(sub), qn, part, nullptr, nr);
                    } else {
                        if (cxd) return cx_dot(st, P, n, (const zd*)W[w0], bp(sub), qn, (double*)part, nullptr, nr, false);
                    }
                    if constexpr (half) {
                        return hipErrorNotSupported;
                    } else {
                        return L::update_dot(st, P, n, (const T*)W[w0], bp(sub), qn, nullptr, nullptr, nullptr, 1, 0,
                                             part, nr, nullptr);
                    }
                });
                run(BGCR_K_SMALL, 0.0, [&] {
                    if constexpr (std::is_same<A, zd>::value) {
                        if (cxd) return cx_reduce(st, (const double*)part, nr, qn * P, P, nullptr, dots + off, nullptr);
                    }
                    return reduce_partials<A>(st, part, nr, nout, nullptr, dots + off, nullptr);
                });
                job.pieces.push_back({w0, wn, q0, qn, off});
                off += nout;
            }
        }
        job.total = off;
        job.valid = true;
        return job;
    }

    // assemble a job's result from a host copy of `dots`
    Mat dot_collect(const DotJob& job, const A* h) const {
        Mat D(job.nq * P, job.nw * P);
        for (const auto& pc : job.pieces)
            for (int wl = 0; wl < pc.wn; ++wl)
                for (int c = 0; c < pc.qn * P; ++c)
                    for (int b = 0; b < P; ++b)
                        D(pc.q0 * P + c, (pc.w0 + wl) * P + b) =
                            to_cd(h[pc.off + (size_t)wl * pc.qn * P * P + (size_t)c * P + b]);
        return D;
    }

    template <class TW>
    Mat multi_dot(const std::vector<const void*>& Q, const std::vector<const TW*>& W) {
        const DotJob job = dot_enqueue(Q, W);
        std::vector<A> h(job.total);
        d2h(h.data(), dots, job.total * sizeof(A));
        return dot_collect(job, h.data());
    }

    // per-column ||B - A X||^2 and ||B||^2 (FP64); stores R (narrowed) if
    // Rout.  residual_enqueue queues the kernel and the copy of its partials
    // to pinned memory; residual_collect waits for them and sums.
    void residual_enqueue(const bgcr_csr* Am, const A* B, int64_t ldb, T* Rout) {
        const double by = (double)(sizeof(A) + 4) * Am->nnz + 4.0 * (n + 1) + 2.0 * sizeof(A) * n * P +
                          (Rout ? (double)sizeof(T) * n * P : 0.0);
        run(BGCR_K_RESIDUAL, by, [&] {
            return residual<A, T>(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, (const A*)Am->values, B, ldb, X, Rout,
                                  dpart, nwg);
        });
        HIPCHK(hipMemcpyAsync(rbuf, dpart, (size_t)nwg * 2 * P * sizeof(double), hipMemcpyDeviceToHost, st));
        if (!ev_res) HIPCHK(hipEventCreateWithFlags(&ev_res, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev_res, st));
        ++n_spmm;
    }
    // waits for the partials only: work queued after them (the refresh
    // combination, the next prologue) keeps the device busy while the host
    // decides and queues the next cycle
    void residual_collect(std::vector<double>& rn2, std::vector<double>& bn2) {
        HIPCHK(hipEventSynchronize(ev_res));
        rn2.assign(P, 0.0);
        bn2.assign(P, 0.0);
        for (int w = 0; w < nwg; ++w)
            for (int b = 0; b < P; ++b) {
                rn2[b] += rbuf[(size_t)w * 2 * P + b];
                bn2[b] += rbuf[(size_t)w * 2 * P + P + b];
            }
    }
    void residual_norms(const bgcr_csr* Am, const A* B, int64_t ldb, T* Rout, std::vector<double>& rn2,
                        std::vector<double>& bn2) {
        residual_enqueue(Am, B, ldb, Rout);
        residual_collect(rn2, bn2);
    }

    // Algorithm 1, U available: A U = C S (CholQR2), U <- U S^{-1}
    void import_basis(const bgcr_csr* Am, const T* avT) {
        const int o = 1 - cur;
        for (int b = 0; b < KB; ++b) {
            // right preconditioning: the operator is A M^{-1}
            if (pc) apply_minv((const T*)ublk(cur, b), nullptr);
            run(BGCR_K_SPMM, (double)(sizeof(T) + 4) * Am->nnz + 4.0 * (n + 1) + 2.0 * sizeof(TB) * n * P, [&] {
                if constexpr (half) {
                    return spmm_block<T, TB, TB, TB>(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, ublk(cur, b),
                                                     nullptr, nullptr, cblk(o, b), nullptr);
                } else {
                    return L::spmm_dot(st, P, n, Am->row_ptr, Am->col_idx, avT, pc ? (const TB*)Zb : ublk(cur, b),
                                       nullptr, nullptr, cblk(o, b), bp({}), 0, 0, part, nwg, nullptr);
                }
            });
            ++n_spmm;
        }
        auto gram_of = [&](int buf) {
            std::vector<const void*> Q;
            std::vector<const TB*> W;
            for (int b = 0; b < KB; ++b) {
                Q.push_back(cblk(buf, b));
                W.push_back(cblk(buf, b));
            }
            return multi_dot(Q, W).block(0, 0, keff, keff);
        };
        Mat S1, S2;
        if (!dense::chol_upper(gram_of(o), S1)) throw Fail{BGCR_ERR_NUMERICAL};
        const Mat S1i = dense::tri_inv_upper(S1);
        std::vector<const void*> inC, inU;
        std::vector<void*> outCcur, outCo, outUo;
        for (int b = 0; b < KB; ++b) {
            inC.push_back(cblk(o, b));
            outCcur.push_back(cblk(cur, b));
        }
        combine<TB>(inC, outCcur, S1i, 0);
        if (!dense::chol_upper(gram_of(cur), S2)) throw Fail{BGCR_ERR_NUMERICAL};
        const Mat S2i = dense::tri_inv_upper(S2);
        inC.clear();
        for (int b = 0; b < KB; ++b) {
            inC.push_back(cblk(cur, b));
            inU.push_back(ublk(cur, b));
            outCo.push_back(cblk(o, b));
            outUo.push_back(ublk(o, b));
        }
        combine<TB>(inC, outCo, S2i, 0);
        const Mat Si = dense::matmul(S1i, S2i);  // S = S2 S1 -> S^{-1} = S1^{-1} S2^{-1}
        combine<TB>(inU, outUo, Si, 0);
        cur = o;
    }

    // X += U C^H R, R -= C C^H R  (Algorithm 1 recycle import, and the start of
    // every refinement step of the precision form)
    void project() {
        std::vector<const void*> Q;
        for (int b = 0; b < KB; ++b) Q.push_back(cblk(cur, b));
        Mat Tm = multi_dot(Q, std::vector<const T*>{R});
        for (int i = keff; i < KP; ++i)
            for (int b = 0; b < P; ++b) Tm(i, b) = 0.0;
        std::vector<const void*> inU, inC;
        for (int b = 0; b < KB; ++b) {
            inU.push_back(ublk(cur, b));
            inC.push_back(cblk(cur, b));
        }
        add_to_X(inU, Tm);
        Mat mT = Tm;
        for (cd& v : mT.a) v = -v;
        combine<T>(inC, {R}, mT, 1);
    }

    // ---- ILU(0) right preconditioning ----------------------------------------
    // (re)allocate a lazily sized device array
    template <class U_>
    void regrow(U_*& ptr, size_t& cap, size_t count) {
        if (count <= cap) return;
        if (ptr) {
            sync();
            (void)hipFree(ptr);
            allocs.erase(std::find(allocs.begin(), allocs.end(), (void*)ptr));
            ptr = nullptr;
            cap = 0;
        }
        ptr = dalloc<U_>(count);
        cap = count;
    }

    // Level schedule of A's pattern, on the host: validated CSR (sorted,
    // in-range columns, a diagonal entry in every row), diagonal positions,
    // and the rows of L and of U ordered by level (a row's level is one more
    // than the largest level among the rows its strictly lower, resp. upper,
    // part refers to).  The pattern is kept on the device to recognise it.
    void ilu_analyse(const bgcr_csr* Am) {
        const int64_t nnz = Am->nnz;
        std::vector<int> rp(n + 1), ci((size_t)nnz);
        d2h(rp.data(), Am->row_ptr, (n + 1) * sizeof(int));
        d2h(ci.data(), Am->col_idx, (size_t)nnz * sizeof(int));
        if (rp[0] != 0 || rp[n] != nnz) throw Fail{BGCR_ERR_INVALID};
        std::vector<int> diag(n), lev(n), ordL, ordU;
        for (int64_t i = 0; i < n; ++i) {
            if (rp[i + 1] < rp[i]) throw Fail{BGCR_ERR_INVALID};
            int d = -1;
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                if (ci[e] < 0 || ci[e] >= n || (e > rp[i] && ci[e] <= ci[e - 1])) throw Fail{BGCR_ERR_INVALID};
                if (ci[e] == i) d = e;
            }
            if (d < 0) throw Fail{BGCR_ERR_INVALID};
            diag[i] = d;
        }
        // rows by level, in increasing index within a level, each level
        // padded with -1 to whole chunks of the single-launch solve
        const int chunk = 256 / P;
        auto order = [&](std::vector<int>& ord, std::vector<int>& ptr) {
            int nl = 0;
            for (int64_t i = 0; i < n; ++i) nl = std::max(nl, lev[i] + 1);
            std::vector<int64_t> cnt(nl, 0);
            for (int64_t i = 0; i < n; ++i) ++cnt[lev[i]];
            ptr.assign(nl + 1, 0);
            for (int l = 0; l < nl; ++l) ptr[l + 1] = ptr[l] + (int)((cnt[l] + chunk - 1) / chunk * chunk);
            ord.assign(ptr[nl], -1);
            std::vector<int> pos(ptr.begin(), ptr.end() - 1);
            for (int64_t i = 0; i < n; ++i) ord[pos[lev[i]]++] = (int)i;
        };
        for (int64_t i = 0; i < n; ++i) {
            int l = 0;
            for (int e = rp[i]; e < diag[i]; ++e) l = std::max(l, lev[ci[e]] + 1);
            lev[i] = l;
        }
        order(ordL, lvlL);
        for (int64_t i = n - 1; i >= 0; --i) {
            int l = 0;
            for (int e = diag[i] + 1; e < rp[i + 1]; ++e) l = std::max(l, lev[ci[e]] + 1);
            lev[i] = l;
        }
        order(ordU, lvlU);
        regrow(d_ci, ci_cap, std::max<size_t>(1, (size_t)nnz));
        regrow(d_ordL, ordL_cap, ordL.size());
        regrow(d_ordU, ordU_cap, ordU.size());
        h2d_big(d_diag, diag.data(), n * sizeof(int));
        h2d_big(d_ordL, ordL.data(), ordL.size() * sizeof(int));
        h2d_big(d_ordU, ordU.data(), ordU.size() * sizeof(int));
        HIPCHK(hipMemcpyAsync(d_rp, Am->row_ptr, (n + 1) * sizeof(int), hipMemcpyDeviceToDevice, st));
        if (nnz > 0)
            HIPCHK(hipMemcpyAsync(d_ci, Am->col_idx, (size_t)nnz * sizeof(int), hipMemcpyDeviceToDevice, st));
        pat_nnz = nnz;
    }

    // larger host -> device copies through the pinned staging buffer
    void h2d_big(void* dst, const void* src, size_t bytes) {
        size_t done = 0;
        while (done < bytes) {
            const size_t c = std::min(bytes - done, hcap);
            sync();
            std::memcpy(hbuf, (const char*)src + done, c);
            HIPCHK(hipMemcpyAsync((char*)dst + done, hbuf, c, hipMemcpyHostToDevice, st));
            done += c;
        }
        sync();
    }

    // Factors of this system: the level schedule (analysed again only when
    // the pattern differs from the last one), then ILU(0) level by level on
    // a copy of A's values.  A zero or non-finite pivot: BGCR_ERR_NUMERICAL.
    void ilu_setup(const bgcr_csr* Am) {
        HostPhase hp(this, BGCR_K_ILU);
        ilu_used = true;
        bool same = false;
        if (pat_nnz == Am->nnz) {
            HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), st));
            HIPCHK(pattern_diff(st, n, Am->nnz, Am->row_ptr, Am->col_idx, d_rp, d_ci, d_flag));
            int f = 1;
            d2h(&f, d_flag, sizeof(int));
            same = f == 0;
        }
        if (!same) ilu_analyse(Am);
        regrow(lu, lu_cap, std::max<size_t>(1, (size_t)Am->nnz));
        if (Am->nnz > 0)
            HIPCHK(hipMemcpyAsync(lu, Am->values, (size_t)Am->nnz * sizeof(A), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), st));
        for (size_t l = 0; l + 1 < lvlL.size(); ++l)
            HIPCHK(ilu0_level<A>(st, d_ordL + lvlL[l], lvlL[l + 1] - lvlL[l], d_rp, d_ci, d_diag, lu, d_flag));
        int f = 0;
        d2h(&f, d_flag, sizeof(int));
        if (f) throw Fail{BGCR_ERR_NUMERICAL};
        // the single-launch solves start from PENDING blocks and zero tickets
        if constexpr (std::is_same<T, A>::value) {
            HIPCHK(fill_pending<T>(st, (int64_t)n * P, Yb));
            HIPCHK(fill_pending<T>(st, (int64_t)n * P, Zb));
        }
        HIPCHK(hipMemsetAsync(d_tick, 0, 2 * sizeof(unsigned), st));
    }

    // a bounded wait of a triangular solve expired during this solve
    bool ilu_wait_expired() {
        int f = 0;
        d2h(&f, d_flag, sizeof(int));
        return f != 0;
    }

    // Zb = M^{-1} in = U^{-1} (L^{-1} in) for a P-column block (in may be Zb):
    // L^{-1} in into Yb, then U^{-1} Yb into Zb, one launch each, each
    // re-arming the other block; skipped on the device while `ctl` says the
    // cycle has stopped
    void apply_minv(const T* in, const Ctl* c) {
        if constexpr (std::is_same<T, A>::value) {
            const double by = (double)(sizeof(A) + 4) * pat_nnz + 4.0 * (n + 1) * 2 + 4.0 * n * 4 +
                              4.0 * sizeof(T) * n * P;
            run(BGCR_K_PRECOND, by, [&] {
                const int64_t nL = lvlL.empty() ? 0 : lvlL.back(), nU = lvlU.empty() ? 0 : lvlU.back();
                HIPCHK(trsv_flow<A>(st, P, true, nL, d_ordL, d_rp, d_ci, d_diag, lu, in, Yb, Zb, d_tick, d_tick + 1,
                                    d_flag, c));
                return trsv_flow<A>(st, P, false, nU, d_ordU, d_rp, d_ci, d_diag, lu, Yb, Zb, Yb, d_tick + 1, d_tick,
                                    d_flag, c);
            });
        } else {
            (void)in;
            (void)c;
            throw Fail{BGCR_ERR_INVALID};
        }
    }

    // X += [in..] K, or with right preconditioning X += M^{-1} ([in..] K): the
    // Krylov and recycled blocks live in the preconditioned variable
    void add_to_X(const std::vector<const void*>& in, const Mat& K) {
        if (!pc) {
            combine<A>(in, {X}, K, 1);
            return;
        }
        combine<A>(in, {(void*)Zb}, K, 0);
        apply_minv(Zb, nullptr);
        combine<A>({(const void*)Zb}, {X}, Mat::eye(P), 1);
    }

    struct CycleOut {
        int meff = 0;
        bool breakdown = false;
        bool has_dots = false;  // refresh dots [U, C, V_1..V_m, V_{m+1}]^H U taken with the cycle
        DotJob spec;            // their layout; the values arrive in dbuf (event ev_dots)
        Mat H, F, Y, RinvLast;
        const void* last = nullptr;  // block holding V_{meff+1} up to RinvLast
    };

    // One restart cycle: CholQR2 of R, m block Arnoldi steps on (I - C C^H) A
    // with BCGS2 + CholQR and the progressive LSQ, then Y (Algorithm 1 loop body).
    // Start of a cycle: cleared H and its triangular factor, and CholQR2 of
    // the starting block R = V_1 Z (Algorithm 1).  Without an enlarged block
    // it needs R only, so plain FP64 queues it before the host solves the
    // previous cycle's refresh.
    void cycle_prologue(bool withC) {
        const int P2 = P * P;
        // H and its triangularised copy are read below the block subdiagonal
        // (block upper Hessenberg structure): those entries must be zero
        const size_t hb = (size_t)(m + 1) * P * m * P * sizeof(A);
        HIPCHK(hipMemsetAsync(H, 0, hb, st));
        HIPCHK(hipMemsetAsync(Rh, 0, hb, st));
        const double blkb = (double)sizeof(T) * n * P;
        const int nr = (use_mx || cx_mx) ? nwg_mx : nwg;
        // Gram partials of the complex matrix-core sweeps are real (2P x 2P)
        auto reduce_gram = [&](A* out) -> hipError_t {
            if constexpr (std::is_same<A, zd>::value) {
                if (cx_mx) return cx_reduce(st, (const double*)part, nr, P, P, nullptr, out, nullptr);
            }
            return reduce_partials<A>(st, part, nr, P2, nullptr, out, nullptr);
        };
        // enlarged block (Section 3.1): the start block is (I - C C^H) [r, Z]
        // with the same L - 1 enlarging vectors Z in every cycle; R's extra
        // columns hold them (the update of R never touches them: Y has one
        // column).  r is orthogonal to C already; the projection of Z takes a
        // dot sweep and an update sweep whose Gram is the first CholQR pass.
        const bool project_z = P > pu && withC && keff > 0;
        if (P > pu) HIPCHK(fill_enlarging<T>(st, R, n, P, pu, 0));
        if (project_z) {
            std::vector<const void*> qc;
            for (int b = 0; b < KB; ++b) qc.push_back(cblk(cur, b));
            const BlockPtrs QC = bp(qc);
            const double cbytes = (double)sizeof(TB) * n * KP;
            run(BGCR_K_TSDOT, blkb + cbytes, [&] {  // T = C^H R
                if constexpr (!std::is_same<T, zd>::value) {
                    if (use_mx) return mfma_dot<T, T, TB>(st, P, n, bp({R}), 1, QC, KB, part, nullptr, nr);
                }
                if constexpr (half) {
                    return hipErrorNotSupported;
                } else {
                    return L::update_dot(st, P, n, R, QC, KB, nullptr, nullptr, nullptr, 1, 0, part, nr, nullptr);
                }
            });
            run(BGCR_K_SMALL, 0.0, [&] {
                HIPCHK(reduce_partials<A>(st, part, nr, KP * P, nullptr, S1, nullptr));
                return zero_cols<A>(st, S1, KP, P, pu);
            });
            run(BGCR_K_TSDOT, 2.0 * blkb + cbytes, [&] {  // R <- R - C T in place, with its Gram
                if constexpr (!std::is_same<T, zd>::value) {
                    if (use_mx) return mfma_proj_gram<T, TB, T>(st, P, n, R, QC, KB, S1, R, part, nullptr, nr);
                }
                if constexpr (half) {
                    return hipErrorNotSupported;
                } else {
                    return L::update_dot(st, P, n, R, QC, KB, S1, nullptr, R, 0, 1, part, nr, nullptr);
                }
            });
        } else {
            run(BGCR_K_TSDOT, blkb, [&] {
                if constexpr (!std::is_same<T, zd>::value) {
                    if (use_mx)
                        return mfma_proj_gram<T, T, T>(st, P, n, R, bp({}), 0, nullptr, nullptr, part, nullptr, nr);
                } else {
                    // the Gram as the dots of R with itself
                    if (cx_mx) return cx_dot(st, P, n, R, bp({R}), 1, (double*)part, nullptr, nr, false);
                }
                return L::update_dot(st, P, n, R, bp({}), 0, nullptr, nullptr, nullptr, 0, 1, part, nr, nullptr);
            });
        }
        run(BGCR_K_SMALL, 0.0, [&] {
            // (after the projection of Z the Gram is that of the sweep's real partials too)
            HIPCHK(project_z ? reduce_partials<A>(st, part, nr, P2, nullptr, Sf, nullptr) : reduce_gram(Sf));
            return cholqr_first<A>(st, P, Sf, Z1, Z1i, pu, ctl);
        });
        const bool cx_second = cx_mx;
        run(BGCR_K_TSDOT, 2.0 * blkb, [&] {
            if constexpr (!std::is_same<T, zd>::value) {
                if (use_mx) {
                    // R Z1^{-1} = R - R (I - Z1^{-1})
                    HIPCHK(i_minus(st, Z1i, S1, P));
                    return mfma_proj_gram<T>(st, P, n, R, bp({R}), 1, S1, W2, part, nullptr, nr);
                }
            } else {
                if (cx_second) {
                    HIPCHK(cx_i_minus(st, Z1i, S1, P));
                    return cx_proj_gram(st, P, n, R, bp({R}), 1, S1, Sr, W2, (double*)part, nullptr, nr, -1);
                }
            }
            return L::update_dot(st, P, n, R, bp({}), 0, nullptr, Z1i, W2, 0, 1, part, nr, nullptr);
        });
        run(BGCR_K_SMALL, 0.0, [&] {
            HIPCHK(cx_second ? reduce_gram(Sf) : reduce_partials<A>(st, part, nr, P2, nullptr, Sf, nullptr));
            return cholqr_second<A>(st, P, Sf, Z1, RinvAll, g, m, pu, ctl);
        });
    }

    // Start block with numerically dependent columns (its CholQR failed): the
    // breakdown rule of the block steps applied to the start block.  A pivoted
    // Cholesky of R's Gram on the host keeps the r independent columns
    // (pivots above 1e-14 of the largest), the other P - r columns become
    // seeded SplitMix64 vectors; the block is projected against C and
    // orthonormalised by CholQR2 into V_1, and the LSQ right-hand side is
    // E V_1^H R.  Real data with the basis in the work type only (false
    // otherwise).  Work buffers: Wb (the block before the first CholQR pass)
    // and W2 (the start block, as the prologue leaves it).
    int deflations = 0;
    bool deflated_prologue(bool withC) {
        if constexpr (std::is_same<T, zd>::value || half) {
            (void)withC;
            return false;
        } else {
            const int P2 = P * P;
            const size_t hb = (size_t)(m + 1) * P * m * P * sizeof(A);
            HIPCHK(hipMemsetAsync(H, 0, hb, st));
            HIPCHK(hipMemsetAsync(Rh, 0, hb, st));
            const double blkb = (double)sizeof(T) * n * P;
            const int nr = use_mx ? nwg_mx : nwg;
            auto gram_only = [&](T* Y) {
                run(BGCR_K_TSDOT, blkb, [&] {
                    if (use_mx) return mfma_proj_gram<T, T, T>(st, P, n, Y, bp({}), 0, nullptr, nullptr, part, nullptr, nr);
                    return L::update_dot(st, P, n, Y, bp({}), 0, nullptr, nullptr, nullptr, 0, 1, part, nr, nullptr);
                });
            };
            gram_only(R);
            run(BGCR_K_SMALL, 0.0, [&] { return reduce_partials<A>(st, part, nr, P2, nullptr, Sf, nullptr); });
            std::vector<A> G(P2);
            d2h(G.data(), Sf, P2 * sizeof(A));
            // pivoted Cholesky G(piv, piv) = R11^T R11 on the leading r columns
            Mat Gm(P, P);
            for (int a = 0; a < P; ++a)
                for (int b = 0; b < P; ++b) Gm(a, b) = to_cd(G[a * P + b]);
            std::vector<int> piv;
            Mat R11m;
            const int r = dense::chol_pivoted(Gm, 1e-14, piv, R11m);
            if (r == 0) return false;
            // T: column c < r of R (Pi R11^{-1}), zero beyond
            const Mat R11i = dense::tri_inv_upper(R11m);
            Mat Tm(P, P);
            for (int a = 0; a < r; ++a)
                for (int c = 0; c < r; ++c) Tm(piv[a], c) = R11i(a, c);
            combine<T>({R}, {Wb}, Tm, 0);
            HIPCHK(fill_enlarging<T>(st, Wb, n, P, r, (uint64_t)(1 + (deflations++ % 200))));
            if (withC && keff > 0) {
                std::vector<const void*> qc;
                for (int b = 0; b < KB; ++b) qc.push_back(cblk(cur, b));
                const BlockPtrs QC = bp(qc);
                const double cbytes = (double)sizeof(TB) * n * KP;
                run(BGCR_K_TSDOT, blkb + cbytes, [&] {
                    if (mx_dot) return mfma_dot<T, T, TB>(st, P, n, bp({Wb}), 1, QC, KB, part, nullptr, nr);
                    return L::update_dot(st, P, n, Wb, QC, KB, nullptr, nullptr, nullptr, 1, 0, part, nr, nullptr);
                });
                run(BGCR_K_SMALL, 0.0, [&] { return reduce_partials<A>(st, part, nr, KP * P, nullptr, S1, nullptr); });
                run(BGCR_K_TSDOT, 2.0 * blkb + cbytes, [&] {  // Wb <- Wb - C T in place, with its Gram
                    if (use_mx) return mfma_proj_gram<T, TB, T>(st, P, n, Wb, QC, KB, S1, Wb, part, nullptr, nr);
                    return L::update_dot(st, P, n, Wb, QC, KB, S1, nullptr, Wb, 0, 1, part, nr, nullptr);
                });
            } else {
                gram_only(Wb);
            }
            run(BGCR_K_SMALL, 0.0, [&] {
                HIPCHK(reduce_partials<A>(st, part, nr, P2, nullptr, Sf, nullptr));
                return cholqr_first<A>(st, P, Sf, Z1, Z1i, r, ctl);
            });
            run(BGCR_K_TSDOT, 2.0 * blkb, [&] {
                if (use_mx) {
                    HIPCHK(i_minus(st, Z1i, S1, P));
                    return mfma_proj_gram<T>(st, P, n, Wb, bp({Wb}), 1, S1, W2, part, nullptr, nr);
                }
                return L::update_dot(st, P, n, Wb, bp({}), 0, nullptr, Z1i, W2, 0, 1, part, nr, nullptr);
            });
            run(BGCR_K_SMALL, 0.0, [&] {
                HIPCHK(reduce_partials<A>(st, part, nr, P2, nullptr, Sf, nullptr));
                return cholqr_second<A>(st, P, Sf, Z1, RinvAll, g, m, P, ctl);
            });
            // right-hand side: V_1^H R = Z2^{-H} (W2^H R), Z2^{-1} = RinvAll[0]
            run(BGCR_K_TSDOT, 2.0 * blkb, [&] {
                if (mx_dot) return mfma_dot<T, T, T>(st, P, n, bp({R}), 1, bp({W2}), 1, part, nullptr, nr);
                return L::update_dot(st, P, n, R, bp({W2}), 1, nullptr, nullptr, nullptr, 1, 0, part, nr, nullptr);
            });
            run(BGCR_K_SMALL, 0.0, [&] { return reduce_partials<A>(st, part, nr, P2, nullptr, S1, nullptr); });
            std::vector<A> hS(P2), hRi0(P2);
            Ctl hc;
            d2h(&hc, ctl, sizeof(Ctl));
            if (hc.active == 0 || hc.status != 0) return false;
            d2h(hS.data(), S1, P2 * sizeof(A));
            d2h(hRi0.data(), RinvAll, P2 * sizeof(A));
            std::vector<A> hg((size_t)(m + 1) * P2, A(0));
            for (int i = 0; i < P; ++i)
                for (int j = 0; j < P; ++j) {
                    double z = 0.0;
                    for (int l = 0; l <= i; ++l) z += hRi0[l * P + i] * hS[l * P + j];  // (Z2^{-1})^T is lower
                    hg[i * P + j] = z;
                }
            h2d(g, hg.data(), hg.size() * sizeof(A));
            return true;
        }
    }

    CycleOut cycle(const bgcr_csr* Am, const T* avT, bool withC, double thresh, bool prologue_done = false,
                   bool deflated = false) {
        const int P2 = P * P;
        if (!prologue_done) cycle_prologue(withC);
        const double sT = (double)sizeof(T), blkb = sT * (double)n * P;
        const double sB = (double)sizeof(TB), vblkb = sB * (double)n * P;  // basis scalar, basis block
        const int ncb = withC ? KB : 0;
        const double kc = withC ? (double)keff : 0.0;
        const double abytes = (sT + 4.0) * (double)Am->nnz + 4.0 * (double)(n + 1);
        // On matrix cores the new block's Gram comes from the second pass
        // (W''^H W'' = W'^H W' - S2^H S2), so its Cholesky factor is known
        // before sweep 3, which then stores V_{j+1} = W'' R_j^{-1} directly;
        // the SpMM of the next step gathers V_{j+1} without normalising.
        const bool pip = pip_order;
        for (int j = 1; j <= m; ++j) {
            cur_step = j;
            std::vector<const void*> Q;
            for (int b = 0; b < ncb; ++b) Q.push_back(cblk(cur, b));
            for (int i = 0; i < j - 1; ++i) Q.push_back(vblk(i));
            const int nq = (int)Q.size();
            const BlockPtrs Q1 = bp(Q);
            const int na = (mx_upd || cx_mx) ? nwg_mx : nwg;
            // sweep 1a: W = A V_j with V_j = W2 R^{-1} (reads A, gathers W2, writes W and V_j)
            // algorithmic bytes per launch follow the byte model of a block step,
            // (s_A + 4) nnz + 4 (n + 1) + 5 s n p + 3 s n q_j: A read and V_j
            // gathered once, W written once and read twice, V_{j+1} written once,
            // Q = [C V_1..V_j] read once per reduction sweep.  This schedule moves
            // two more blocks per step than the model (the first dots re-read W,
            // and W'' is stored raw then normalised in the next SpMM); they are
            // not counted.  SpMM: A, V_j, W.
            // Off the PIP order (W'' stored raw) V_j = W2 R_{j-1}^{-1} is stored
            // before the SpMM, which then forms A V_j from the stored block:
            // (A W2) R^{-1} would satisfy the Arnoldi relation only to rounding
            // times cond(R_{j-1}), which an almost rank-deficient block makes
            // large (complex Helmholtz: |A U - C| / |C| 1e-10 against the
            // oracle's 5e-14).  Step 1 off the fused sweep keeps the scaled
            // SpMM: its factor is the second CholQR2 pass, close to the identity.
            const bool norm_first = std::is_same<T, A>::value && !pip && j > 1 && P > 1;
            // sweeps 1a and 1b in one pass (FP64 on matrix cores): from step 2
            // V_j is stored, normalised, by the previous step's third sweep; at
            // step 1, V_1 = W2 R^{-1} is stored first
            std::vector<const void*> Qd(Q);
            Qd.push_back(vblk(j - 1));
            const double qbytes = sB * n * (kc + (double)j * P);
            const bool fused = fuse_dots && pip && ((int)Qd.size() * P + 15) / 16 <= 12;
            if constexpr (std::is_same<T, A>::value) {
                if (pc || norm_first || (fused && j == 1)) {
                    // V_j as a stored block (off matrix cores, and at j = 1, it
                    // is W2 R^{-1}); with a preconditioner then M^{-1} V_j into
                    // Zb, which the SpMM reads
                    if (!(pip && j > 1))
                        run(BGCR_K_COMBINE, vblkb + blkb, [&] {
                            return rows_times<T>(st, P, n, (const T*)W2, RinvAll + (size_t)(j - 1) * P2,
                                                 (T*)vblk(j - 1), ctl);
                        });
                    if (pc) apply_minv((const T*)vblk(j - 1), ctl);
                }
            }
            if (fused) {
                run(BGCR_K_ARN_SPMM_DOT, abytes + vblkb + blkb + qbytes, [&] {
                    if constexpr (std::is_same<T, double>::value && !half) {
                        return spmm_dot_mfma(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT,
                                             pc ? (const T*)Zb : (const T*)vblk(j - 1), Wb, bp(Qd), (int)Qd.size(),
                                             part, ctl);
                    }
                    return hipErrorNotSupported;
                });
            } else run(BGCR_K_ARN_SPMM, abytes + vblkb + blkb, [&] {
                if constexpr (half) {
                    if (j > 1)
                        return spmm_block<T, TB, TB, T>(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, vblk(j - 1),
                                                        nullptr, nullptr, Wb, ctl);
                    return spmm_block<T, T, TB, T>(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, W2, RinvAll,
                                                   vblk(0), Wb, ctl);
                } else {
                    if (pc)
                        return L::spmm_rinv(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, Zb, nullptr, nullptr, Wb,
                                            ctl);
                    if ((pip || norm_first) && j > 1)
                        return L::spmm_rinv(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, vblk(j - 1), nullptr,
                                            nullptr, Wb, ctl);
                    return L::spmm_rinv(st, P, n, Am->nnz, Am->row_ptr, Am->col_idx, avT, W2,
                                        RinvAll + (size_t)(j - 1) * P2, vblk(j - 1), Wb, ctl);
                }
            });
            Q.push_back(vblk(j - 1));
            const BlockPtrs QB = bp(Q);
            // sweep 1b: first block-CGS dots [C V_1..V_j]^H W (reads W and Q)
            // one-column blocks take the streaming P = 1 sweeps (up to 32 blocks)
            const bool narrow = !std::is_same<T, zd>::value && !half && P == 1 && nq + 1 <= 32;
            if (!fused) run(BGCR_K_ARN_DOT, qbytes, [&] {  // Q
                if constexpr (!std::is_same<T, zd>::value && !half) {
                    if (narrow) return narrow_sweep<T>(st, n, Wb, QB, nq + 1, nullptr, nullptr, part, na, ctl, true);
                }
                if constexpr (!std::is_same<T, zd>::value) {
                    if (mx_dot) return mfma_dot<T, T, TB>(st, P, n, bp({Wb}), 1, QB, nq + 1, part, ctl, na, alt_dir && pip);
                } else {
                    if (cx_mx) return cx_dot(st, P, n, Wb, QB, nq + 1, (double*)part, ctl, na, alt_dir && pip);
                }
                return L::update_dot(st, P, n, Wb, QB, nq + 1, nullptr, nullptr, nullptr, 1, 0, part, na, ctl, 0);
            });
            const int nout = (nq + 1) * P2;
            const int nd = fused ? spmm_dot_nwg(P, n) : na;
            run(BGCR_K_SMALL, 0.0, [&] {
                if constexpr (std::is_same<A, zd>::value) {
                    if (cx_mx) return cx_reduce(st, (const double*)part, nd, (nq + 1) * P, P, nullptr, S1, ctl);
                }
                return reduce_partials<A>(st, part, nd, nout, nullptr, S1, ctl);
            });
            run(BGCR_K_PROJ_DOT, blkb + qbytes, [&] {  // W, Q
                if constexpr (!std::is_same<T, zd>::value && !half) {
                    if (narrow) return narrow_sweep<T>(st, n, Wb, QB, nq + 1, S1, nullptr, part, na, ctl, true);
                }
                if constexpr (!std::is_same<T, zd>::value) {
                    if (mx_upd)
                        return mfma_proj_dot<T, TB>(st, P, n, Wb, QB, nq + 1, S1, part, ctl, na, pip,
                                                    alt_dir && fused);
                } else {
                    // (P = 16 with more than 10 blocks in Q stores W' in W2, which
                    // the SpMM has consumed)
                    if (cx_mx)
                        return cx_proj_dot(st, P, n, Wb, QB, nq + 1, S1, Sr, W2, (double*)part, ctl, na, pip, false);
                }
                return L::update_dot(st, P, n, Wb, QB, nq + 1, S1, nullptr, nullptr, 1, 0, part, na, ctl, 1);
            });
            if (pip) {
                run(BGCR_K_SMALL, 0.0, [&] {
                    bool done = false;
                    if constexpr (std::is_same<A, zd>::value) {
                        if (cx_mx) {
                            // real partials [dots 4 q P | Gram 4 P P] per workgroup
                            const int64_t qd = (int64_t)(nq + 1) * P, stride = 4 * qd * P + 4 * (int64_t)P2;
                            HIPCHK(cx_reduce_at(st, (const double*)part, na, stride, 0, (int)qd, P, S1, Sf, ctl));
                            HIPCHK(cx_reduce_at(st, (const double*)part, na, stride, 4 * qd * P, P, P, nullptr,
                                                Sf + nout, ctl));
                            done = true;
                        }
                    }
                    if (!done) HIPCHK(reduce_partials<A>(st, part, na, nout + P2, S1, Sf, ctl, nout));
                    return step_small<A>(st, P, Sf + nout, Sf, S1, ncb * P, j, m, H, F, Rh, QH, g, RinvAll, rho, ctl,
                                         thresh);
                });
                run(BGCR_K_PROJ_GRAM, blkb + vblkb + qbytes, [&] {  // W, V_{j+1}, Q
                    if constexpr (!std::is_same<T, zd>::value) {
                        return mfma_proj_gram<T, TB, TB>(st, P, n, Wb, QB, nq + 1, Sf, vblk(j), part, ctl, na,
                                                         (const double*)(RinvAll + (size_t)j * P2), j,
                                                         alt_dir && !fused);
                    } else {
                        return cx_proj_norm(st, P, n, Wb, QB, nq + 1, Sf, Sr, RinvAll + (size_t)j * P2, vblk(j),
                                            (double*)part, ctl, na, j, alt_dir);
                    }
                });
                continue;
            }
            run(BGCR_K_SMALL, 0.0, [&] {
                if constexpr (std::is_same<A, zd>::value) {
                    if (cx_mx) return cx_reduce(st, (const double*)part, na, (nq + 1) * P, P, S1, Sf, ctl);
                }
                return reduce_partials<A>(st, part, na, nout, S1, Sf, ctl);
            });
            run(BGCR_K_PROJ_GRAM, 2.0 * blkb + qbytes, [&] {  // W, V_{j+1}, Q
                if constexpr (!std::is_same<T, zd>::value && !half) {
                    if (narrow) return narrow_sweep<T>(st, n, Wb, QB, nq + 1, Sf, W2, part, na, ctl, false);
                }
                if constexpr (!std::is_same<T, zd>::value) {
                    if (mx_upd) return mfma_proj_gram<T>(st, P, n, Wb, QB, nq + 1, Sf, W2, part, ctl, na);
                } else {
                    if (cx_mx) return cx_proj_gram(st, P, n, Wb, QB, nq + 1, Sf, Sr, W2, (double*)part, ctl, na, j);
                }
                return L::update_dot(st, P, n, Wb, QB, nq + 1, Sf, nullptr, W2, 0, 1, part, na, ctl, 2);
            });
            run(BGCR_K_SMALL, 0.0, [&] {
                if constexpr (std::is_same<A, zd>::value) {
                    if (cx_mx) HIPCHK(cx_reduce(st, (const double*)part, na, P, P, nullptr, S1, ctl));
                    else HIPCHK(reduce_partials<A>(st, part, na, P2, nullptr, S1, ctl));
                } else {
                    HIPCHK(reduce_partials<A>(st, part, na, P2, nullptr, S1, ctl));
                }
                return step_small<A>(st, P, S1, Sf, nullptr, ncb * P, j, m, H, F, Rh, QH, g, RinvAll, rho, ctl, thresh);
            });
        }
        cur_step = 0;
        // The refresh after this cycle needs [U, C, V_1..V_meff, V_{meff+1}]^H U;
        // every cycle but a system's last runs all m steps without breakdown,
        // so the dots are taken now, with V_{m+1} = W'' R^{-1}, and arrive with
        // the cycle's small results in one copy (redone by the refresh when the
        // guess was wrong).
        // Off the PIP order V_{m+1} = W'' R_m^{-1} is stored like the other
        // blocks (see norm_first) and becomes the cycle's last block; when the
        // cycle stopped earlier, the block of that step is stored after the
        // copy below.
        const bool norm_last = std::is_same<T, A>::value && !pip && P > 1;
        if constexpr (std::is_same<T, A>::value) {
            if (norm_last)
                run(BGCR_K_COMBINE, vblkb + blkb, [&] {
                    return rows_times<T>(st, P, n, (const T*)W2, RinvAll + (size_t)m * P2, (T*)vblk(m), nullptr);
                });
        }
        // The steps' results are copied back first and the dots after them, into
        // a buffer of their own: the host reads the results and queues the
        // solution update while the dots run, and waits for the dots only when
        // the refresh needs them.  (Stream order puts the first copy after
        // every staged upload that reads hbuf; nothing is staged between the
        // copy and its event.)
        HIPCHK(hipMemcpyAsync(hbuf, hr, off_dots, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(ev_cyc, st));
        DotJob spec;
        if (withC && k > 0) {
            std::vector<const void*> Qs;
            std::vector<const TB*> Ws;
            for (int b = 0; b < KB; ++b) Qs.push_back(ublk(cur, b));
            for (int b = 0; b < KB; ++b) Qs.push_back(cblk(cur, b));
            for (int i = 0; i < m; ++i) Qs.push_back(vblk(i));
            Qs.push_back((pip || norm_last) ? (const void*)vblk(m) : (const void*)W2);
            for (int b = 0; b < KB; ++b) Ws.push_back(ublk(cur, b));
            spec = dot_enqueue(Qs, Ws);
            HIPCHK(hipMemcpyAsync(dbuf, dots, spec.total * sizeof(A), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(ev_dots, st));
        }
        HIPCHK(hipEventSynchronize(ev_cyc));
        hoff = 0;
        Ctl hc;
        std::memcpy(&hc, hbuf, sizeof(Ctl));
        const A* hH = (const A*)(hbuf + off_H);
        const A* hR = (const A*)(hbuf + off_Rh);
        const A* hg = (const A*)(hbuf + off_g);
        const A* hRi = (const A*)(hbuf + off_Ri);
        const A* hF = (const A*)(hbuf + off_F);
        CycleOut co;
        co.meff = hc.meff;
        co.breakdown = hc.status != 0;
        if (co.meff == 0) {
            // the start block was rank deficient: one retry with a deflated start block
            if (deflated || !deflated_prologue(withC)) throw Fail{BGCR_ERR_NUMERICAL};
            ++n_deflated;
            return cycle(Am, avT, withC, thresh, true, true);
        }
        const int me = co.meff, mp = me * P, ldH = m * P;
        HostPhase hp(this, BGCR_K_HOST);
        if (spec.valid && me == m && !co.breakdown) {
            co.spec = spec;
            co.has_dots = true;
        }
        co.H = Mat((me + 1) * P, mp);
        for (int i = 0; i < (me + 1) * P; ++i)
            for (int j = 0; j < mp; ++j) co.H(i, j) = to_cd(hH[(size_t)i * ldH + j]);
        Mat Rt(mp, mp), gt(mp, P);
        for (int i = 0; i < mp; ++i) {
            for (int j = 0; j < mp; ++j) Rt(i, j) = to_cd(hR[(size_t)i * ldH + j]);
            for (int b = 0; b < P; ++b) gt(i, b) = to_cd(hg[(size_t)i * P + b]);
        }
        co.Y = dense::solve_upper(Rt, gt);
        co.F = Mat(withC ? KP : 0, mp);
        if (withC)
            for (int i = 0; i < KP; ++i)
                for (int j = 0; j < mp; ++j) co.F(i, j) = to_cd(hF[(size_t)i * ldH + j]);
        co.RinvLast = Mat(P, P);
        if (pip) {
            // V_{meff+1} was stored normalised by sweep 3 of step meff (or of the last good step)
            co.last = vblk(me);
            co.RinvLast = Mat::eye(P);
        } else if (co.breakdown) {
            // step meff+1 failed its Cholesky: V_{meff+1} is the normalised block in slot meff
            co.last = vblk(me);
            co.RinvLast = Mat::eye(P);
        } else if (norm_last) {
            if constexpr (std::is_same<T, A>::value) {
                if (me < m)
                    HIPCHK(rows_times<T>(st, P, n, (const T*)W2, RinvAll + (size_t)me * P2, (T*)vblk(me), nullptr));
            }
            co.last = vblk(me);
            co.RinvLast = Mat::eye(P);
        } else {
            co.last = W2;
            for (int a = 0; a < P; ++a)
                for (int b = 0; b < P; ++b) co.RinvLast(a, b) = to_cd(hRi[(size_t)me * P2 + a * P + b]);
        }
        if (co.breakdown) ++n_deflated;
        if (prof) prof_resolve(hc.meff);
        // model-M algorithmic bytes of the executed Arnoldi sweeps: V_j
        // gathered and V_{j+1} written in the basis type, W written once and
        // read twice in the work type, Q read once per reduction sweep
        for (int j = 1; j <= me; ++j)
            alg_bytes += abytes + 2.0 * vblkb + 3.0 * blkb + 3.0 * sB * n * (kc + (double)j * P);
        n_spmm += me;
        n_steps += me;
        return co;
    }

    // X += W_m Y - U F Y ; (plain) R -= W_{m+1} H Y  (Algorithm 1)
    void update_solution(const CycleOut& co, bool withC, bool update_R) {
        const int me = co.meff, mp = me * P;
        if constexpr (std::is_same<T, A>::value) {
            if (update_R && !pc) {
                // both in one pass over the basis: [X, R] += [V_1..V_me, U, V_{me+1}] K
                std::vector<const void*> in2;
                for (int i = 0; i < me; ++i) in2.push_back(vblk(i));
                const int nu = withC ? KB : 0;
                for (int b = 0; b < nu; ++b) in2.push_back(ublk(cur, b));
                in2.push_back(co.last);
                const int rows = mp + nu * P + P;
                Mat K2(rows, 2 * P);
                Mat HY = dense::matmul(co.H, co.Y);
                Mat last = dense::matmul(co.RinvLast, HY.block(mp, 0, P, P));
                for (int i = 0; i < mp; ++i)
                    for (int b = 0; b < P; ++b) {
                        K2(i, b) = co.Y(i, b);
                        K2(i, P + b) = -HY(i, b);
                    }
                if (withC) {
                    Mat FY = dense::matmul(co.F, co.Y);
                    for (int i = 0; i < keff; ++i)
                        for (int b = 0; b < P; ++b) K2(mp + i, b) = -FY(i, b);
                }
                for (int i = 0; i < P; ++i)
                    for (int b = 0; b < P; ++b) K2(mp + nu * P + i, P + b) = -last(i, b);
                combine<A>(in2, {(void*)X, (void*)R}, K2, 2);
                return;
            }
        }
        std::vector<const void*> in;
        for (int i = 0; i < me; ++i) in.push_back(vblk(i));
        Mat KX(mp + (withC ? KP : 0), P);
        KX.set_block(0, 0, co.Y);
        if (withC) {
            Mat FY = dense::matmul(co.F, co.Y);
            for (cd& v : FY.a) v = -v;
            for (int i = keff; i < KP; ++i)
                for (int b = 0; b < P; ++b) FY(i, b) = 0.0;
            KX.set_block(mp, 0, FY);
            for (int b = 0; b < KB; ++b) in.push_back(ublk(cur, b));
        }
        add_to_X(in, KX);
        if (update_R) {
            Mat HY = dense::matmul(co.H, co.Y);
            Mat KR((me + 1) * P, P);
            for (int i = 0; i < mp; ++i)
                for (int b = 0; b < P; ++b) KR(i, b) = -HY(i, b);
            Mat last = dense::matmul(co.RinvLast, HY.block(mp, 0, P, P));
            for (int i = 0; i < P; ++i)
                for (int b = 0; b < P; ++b) KR(mp + i, b) = -last(i, b);
            std::vector<const void*> inR;
            for (int i = 0; i < me; ++i) inR.push_back(vblk(i));
            inR.push_back(co.last);
            combine<T>(inR, {R}, KR, 1);
        }
    }

    // basis of the selected harmonic Ritz vectors: columns t (complex), or
    // [Re t, Im t] / Re t for real problems
    void ritz_basis(const dense::Selection& sel, const std::vector<std::vector<cd>>& vecs, Mat& Pm) {
        const int dim = vecs.empty() ? 0 : (int)vecs[0].size();
        Pm = Mat(dim, sel.ncols);
        int col = 0;
        for (size_t s = 0; s < sel.idx.size(); ++s) {
            const std::vector<cd>& t = vecs[s];
            if (cplx) {
                for (int i = 0; i < dim; ++i) Pm(i, col) = t[i];
                ++col;
            } else if (sel.pair_first[s]) {
                for (int i = 0; i < dim; ++i) {
                    Pm(i, col) = t[i].real();
                    Pm(i, col + 1) = t[i].imag();
                }
                col += 2;
            } else {
                int jm = 0;
                for (int i = 1; i < dim; ++i)
                    if (std::abs(t[i]) > std::abs(t[jm])) jm = i;
                const cd ph = std::abs(t[jm]) > 0 ? std::conj(t[jm]) / std::abs(t[jm]) : cd(1.0, 0.0);
                for (int i = 0; i < dim; ++i) Pm(i, col) = (t[i] * ph).real();
                ++col;
            }
        }
    }

    // Eigenvalues of K, harmonic Ritz values theta (theta = 1/mu when `inverse`),
    // selection, and the selected eigenvectors.  `robust` uses the full Schur
    // form (fallback when inverse iteration gives nearly dependent vectors).
    void eig_select(const Mat& K, bool inverse, int kt, bool robust, std::vector<cd>& theta, dense::Selection& sel,
                    std::vector<std::vector<cd>>& vecs) {
        HostPhase hp(this, BGCR_K_HOST_EIG);
        const int nn = K.r;
        theta.assign(nn, cd(0.0, 0.0));
        vecs.clear();
        auto to_theta = [&](cd mu) { return !inverse ? mu : (std::abs(mu) > 0.0 ? 1.0 / mu : cd(INFINITY, 0.0)); };
        if (!robust) {
            dense::EigSolver E;
            E.compute(K, !cplx);
            if (E.ok) {
                for (int i = 0; i < nn; ++i) theta[i] = to_theta(E.lam[i]);
                sel = dense::select_ritz(theta, kt, prm.select_largest != 0, !cplx);
                vecs = E.vectors_for(sel.idx);
                return;
            }
        }
        dense::Schur S = dense::schur(K);
        if (!S.ok) throw Fail{BGCR_ERR_NUMERICAL};
        for (int i = 0; i < nn; ++i) theta[i] = to_theta(S.lam[i]);
        sel = dense::select_ritz(theta, kt, prm.select_largest != 0, !cplx);
        for (int i : sel.idx) vecs.push_back(dense::schur_eigvec(S, i));
    }

    // The triangular factor rho of G P is inverted into the coefficients of U
    // (U = [..] P rho^{-1}): rounding in forming U reaches A U - C amplified by
    // about cond(rho).  Inverse iteration can return nearly dependent vectors
    // for clustered harmonic Ritz values (P, hence rho, ill-conditioned while
    // the eigenvectors themselves are not: complex Helmholtz, p = 16, gave
    // cond(rho) near 1e5 and |A U - C| / |C| = 1e-10 against the oracle's
    // 4e-15); the refresh then takes the vectors from the Schur form.
    static bool well_conditioned_r(const Mat& r) {
        const int k = std::min(r.r, r.c);
        double mx = 0.0, mn = INFINITY;
        for (int i = 0; i < k; ++i) {
            mx = std::max(mx, std::abs(r(i, i)));
            mn = std::min(mn, std::abs(r(i, i)));
        }
        if (!(mx > 0.0 && mn > 1e-10 * mx)) return false;
        // 1-norm condition number of the square leading part
        Mat sq(k, k);
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= j; ++i) sq(i, j) = r(i, j);
        const Mat ri = dense::tri_inv_upper(sq);
        double n1 = 0.0, ni = 0.0;
        for (int j = 0; j < k; ++j) {
            double a = 0.0, b = 0.0;
            for (int i = 0; i < k; ++i) {
                a += std::abs(sq(i, j));
                b += std::abs(ri(i, j));
            }
            n1 = std::max(n1, a);
            ni = std::max(ni, b);
        }
        return n1 * ni <= 1e4;
    }

    // The refresh of (U, C) as one block combination: outputs = inputs K
    struct RefreshPlan {
        bool active = false;
        std::vector<const void*> in;
        std::vector<void*> out;
        Mat K;
        int kn = 0;
        int next_cur = 0;
    };

    void apply_refresh(const RefreshPlan& rp) {
        combine<TB>(rp.in, rp.out, rp.K, 0);
        cur = rp.next_cur;
        keff = rp.kn;
    }

    // first system, no U (Algorithm 1 else-branch): Proposition block-harm-ritz
    void refresh_first(const CycleOut& co, RefreshPlan& rp) {
        const int me = co.meff, mp = me * P;
        const int kt = std::min(k, mp);
        if (kt == 0) {
            keff = 0;
            return;
        }
        std::unique_ptr<HostPhase> hp(new HostPhase(this, BGCR_K_HOST));
        Mat Hm = co.H.block(0, 0, mp, mp);
        Mat Hs = co.H.block(mp, mp - P, P, P);
        Mat rhs(mp, P);
        rhs.set_block(mp - P, 0, dense::matmul(dense::adjoint(Hs), Hs));
        Mat Xs;
        Mat K = Hm;
        std::vector<cd> theta;
        std::vector<std::vector<cd>> vecs;
        dense::Selection sel;
        Mat Pm, Qg, rg;
        // Ritz vectors (Section 4.1.3): eigenvectors of H_m = W_m^H A W_m itself
        const bool ritz = prm.ritz_vectors != 0;
        const bool standard = ritz || dense::solve_lu(dense::adjoint(Hm), rhs, Xs);
        if (standard && !ritz)
            for (int i = 0; i < mp; ++i)
                for (int b = 0; b < P; ++b) K(i, mp - P + b) += Xs(i, b);
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (standard) {
                eig_select(K, false, kt, attempt == 1, theta, sel, vecs);
            } else {
                // singular H_m: generalized form with no recycled space
                Mat M(co.H.r, mp);
                for (int i = 0; i < mp; ++i) M(i, i) = 1.0;
                gen_harmonic(co.H, M, kt, theta, sel, vecs, attempt == 1);
            }
            ritz_basis(sel, vecs, Pm);
            dense::qr_pos(dense::matmul(co.H, Pm), Qg, rg);
            if (well_conditioned_r(rg)) break;
        }
        const int kn = Pm.c;
        if (kn > KP) throw Fail{BGCR_ERR_NUMERICAL};
        Mat PR = dense::matmul(Pm, dense::tri_inv_upper(rg));
        // inputs [V_1..V_meff, last]; outputs [U blocks, C blocks]
        Mat K2((me + 1) * P, 2 * KP);
        for (int i = 0; i < mp; ++i)
            for (int c = 0; c < kn; ++c) {
                K2(i, c) = PR(i, c);
                K2(i, KP + c) = Qg(i, c);
            }
        Mat lastQ = dense::matmul(co.RinvLast, Qg.block(mp, 0, P, kn));
        for (int i = 0; i < P; ++i)
            for (int c = 0; c < kn; ++c) K2(mp + i, KP + c) = lastQ(i, c);
        std::vector<const void*> in;
        for (int i = 0; i < me; ++i) in.push_back(vblk(i));
        in.push_back(co.last);
        std::vector<void*> out;
        for (int b = 0; b < KB; ++b) out.push_back(ublk(cur, b));
        for (int b = 0; b < KB; ++b) out.push_back(cblk(cur, b));
        rp.active = true;
        rp.in = in;
        rp.out = out;
        rp.K = K2;
        rp.kn = kn;
        rp.next_cur = cur;
    }

    // harmonic Ritz on the augmented space, eq. harm-ritz-gen-eig:
    // G^H G t = theta G^H M t  with G = Qg Rg:  (Qg^H M Rg^{-1}) s = mu s,
    // theta = 1/mu, t = Rg^{-1} s.  G = [[D, F], [0, H_m]] (or H_m) has lower
    // bandwidth P: D is diagonal and the subdiagonal blocks R_j of the block
    // Hessenberg H_m are upper triangular.
    // QR of G (lower bandwidth p) and the inverse of its triangular factor
    struct GFactor {
        Mat Qg, Rgi;
    };
    GFactor factor_g(const Mat& G) {
        GFactor f;
        Mat Rg;
        dense::qr_pos(G, f.Qg, Rg, P);
        for (int i = 0; i < G.c; ++i)
            if (!(std::abs(Rg(i, i)) > 0.0)) throw Fail{BGCR_ERR_NUMERICAL};
        f.Rgi = dense::tri_inv_upper(Rg);
        return f;
    }

    void gen_harmonic(const Mat& G, const Mat& M, int kt, std::vector<cd>& theta, dense::Selection& sel,
                      std::vector<std::vector<cd>>& vecs, bool robust) {
        gen_harmonic(factor_g(G), M, nullptr, kt, theta, sel, vecs, robust);
    }

    // With `colscale`, G = G' diag(colscale^{-1}, 1, ..) is given by the factors
    // of G' and M by M diag(colscale, 1, ..) (its leading columns unscaled):
    // K is the same matrix, and t = diag(colscale, 1, ..) R'^{-1} s.
    void gen_harmonic(const GFactor& gf, const Mat& M, const std::vector<double>* colscale, int kt,
                      std::vector<cd>& theta, dense::Selection& sel, std::vector<std::vector<cd>>& vecs, bool robust) {
        const Mat& Qg = gf.Qg;
        const Mat& Rgi = gf.Rgi;
        const int nn = Rgi.c;
        // K = Qg^H M Rg^{-1}.  The columns of M that are unit vectors e_r (its
        // identity block W_{m+1}^H W_m) give row r of Qg, conjugated, without a
        // product; the rest are dot products.  Rg^{-1} is upper triangular.
        const int rows = M.r, mc = M.c;
        std::vector<int> unit_row(mc, -1);
        std::vector<int> dense_cols;
        for (int c = 0; c < mc; ++c) {
            int r1 = -1, nz = 0;
            for (int r = 0; r < rows && nz < 2; ++r)
                if (M(r, c) != cd(0.0, 0.0)) {
                    ++nz;
                    r1 = r;
                }
            if (nz == 1 && M(r1, c) == cd(1.0, 0.0))
                unit_row[c] = r1;
            else
                dense_cols.push_back(c);
        }
        Mat K1(nn, mc);
        for (int c = 0; c < mc; ++c)
            if (unit_row[c] >= 0)
                for (int i = 0; i < nn; ++i) K1(i, c) = std::conj(Qg(unit_row[c], i));
        if (!dense_cols.empty()) {
            Mat Md(rows, (int)dense_cols.size());
            for (int j = 0; j < (int)dense_cols.size(); ++j)
                for (int r = 0; r < rows; ++r) Md(r, j) = M(r, dense_cols[j]);
            const Mat Kd = dense::matmul(dense::adjoint(Qg), Md);
            for (int j = 0; j < (int)dense_cols.size(); ++j)
                for (int i = 0; i < nn; ++i) K1(i, dense_cols[j]) = Kd(i, j);
        }
        const Mat K = dense::matmul_upper(K1, Rgi);
        std::vector<std::vector<cd>> svecs;
        eig_select(K, true, kt, robust, theta, sel, svecs);
        vecs.clear();
        for (const auto& sv : svecs) {
            std::vector<cd> tv(nn, cd(0.0, 0.0));
            for (int r = 0; r < nn; ++r)
                for (int c = r; c < nn; ++c) tv[r] += Rgi(r, c) * sv[c];
            if (colscale)
                for (size_t r = 0; r < colscale->size(); ++r) tv[r] *= (*colscale)[r];
            vecs.push_back(tv);
        }
    }

    // Ritz pairs of the pencil (Ah, Bh), Bh Hermitian positive definite:
    // Bh = Rb^H Rb, eigenpairs (theta, s) of Rb^{-H} Ah Rb^{-1}, t = Rb^{-1} s
    void gen_ritz(const Mat& Ah, const Mat& Bh, int kt, std::vector<cd>& theta, dense::Selection& sel,
                  std::vector<std::vector<cd>>& vecs, bool robust) {
        Mat Rb;
        if (!dense::chol_upper(Bh, Rb)) throw Fail{BGCR_ERR_NUMERICAL};
        const Mat Rbi = dense::tri_inv_upper(Rb);
        const Mat K = dense::matmul(dense::matmul(dense::adjoint(Rbi), Ah), Rbi);
        std::vector<std::vector<cd>> svecs;
        eig_select(K, false, kt, robust, theta, sel, svecs);
        const int nn = Ah.c;
        vecs.clear();
        for (const auto& sv : svecs) {
            std::vector<cd> tv(nn, cd(0.0, 0.0));
            for (int r = 0; r < nn; ++r)
                for (int c = r; c < nn; ++c) tv[r] += Rbi(r, c) * sv[c];
            vecs.push_back(tv);
        }
    }

    // Algorithm 1, end of a cycle with recycling: D, G_m, harmonic Ritz on
    // U + K_m, then C <- [C W_{m+1}] Q, U <- [U D  W_m] P rho^{-1}
    void refresh_aug(const CycleOut& co, RefreshPlan& rp) {
        const int me = co.meff, mp = me * P;
        // dots [U, C, V_1..V_meff, last]^H U
        std::vector<const void*> Q;
        std::vector<const TB*> W;
        for (int b = 0; b < KB; ++b) Q.push_back(ublk(cur, b));
        for (int b = 0; b < KB; ++b) Q.push_back(cblk(cur, b));
        for (int i = 0; i < me; ++i) Q.push_back(vblk(i));
        Q.push_back(co.last);
        for (int b = 0; b < KB; ++b) W.push_back(ublk(cur, b));
        const int ke = keff;
        const int rows = ke + (me + 1) * P, cols = ke + mp;
        const bool harmonic = !prm.ritz_vectors;
        // G = [D F; 0 H] = [I F; 0 H] diag(D, I) with D = diag(1 / |u_i|): the
        // QR of the first factor needs no dots, so it is taken while they are
        // on their way (the harmonic problem then uses M diag(D^{-1}, I))
        GFactor gf;
        if (harmonic) {
            HostPhase hp0(this, BGCR_K_HOST);
            Mat G1(rows, cols);
            for (int i = 0; i < ke; ++i) G1(i, i) = 1.0;
            for (int i = 0; i < ke; ++i)
                for (int j = 0; j < mp; ++j) G1(i, ke + j) = co.F(i, j);
            G1.set_block(ke, ke, co.H);
            gf = factor_g(G1);
        }
        Mat Dm;
        if (co.has_dots) {
            HIPCHK(hipEventSynchronize(ev_dots));
            Dm = dot_collect(co.spec, dbuf);
        } else {
            Dm = multi_dot(Q, W);
        }
        std::unique_ptr<HostPhase> hp(new HostPhase(this, BGCR_K_HOST));
        std::vector<double> d(ke), unorm(ke);
        for (int i = 0; i < ke; ++i) {
            const double nu = std::sqrt(std::max(Dm(i, i).real(), 0.0));
            if (!(nu > 0.0)) throw Fail{BGCR_ERR_NUMERICAL};
            unorm[i] = nu;
            d[i] = 1.0 / nu;
        }
        Mat G(rows, cols), M(rows, cols);
        for (int i = 0; i < ke; ++i) G(i, i) = d[i];
        for (int i = 0; i < ke; ++i)
            for (int j = 0; j < mp; ++j) G(i, ke + j) = co.F(i, j);
        G.set_block(ke, ke, co.H);
        // M = [C W_{m+1}]^H [U D  W_m] using C^H W = 0 and W^H W = I (for the
        // harmonic problem with its leading columns unscaled, M diag(D^{-1}, I))
        auto msc = [&](int j) { return harmonic ? 1.0 : d[j]; };
        for (int i = 0; i < ke; ++i)
            for (int j = 0; j < ke; ++j) M(i, j) = Dm(KP + i, j) * msc(j);
        for (int i = 0; i < mp; ++i)
            for (int j = 0; j < ke; ++j) M(ke + i, j) = Dm(2 * KP + i, j) * msc(j);
        Mat WlU = Dm.block(2 * KP + mp, 0, P, ke);
        Mat VlU = dense::matmul(dense::adjoint(co.RinvLast), WlU);
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < ke; ++j) M(ke + mp + i, j) = VlU(i, j) * msc(j);
        for (int i = 0; i < mp; ++i) M(ke + i, ke + i) = 1.0;
        const int kt = std::min(k, cols);
        std::vector<cd> theta;
        dense::Selection sel;
        std::vector<std::vector<cd>> vecs;
        Mat Pm, Qg, rg;
        // Ritz vectors (Section 4.1.3): What = [U D  W_m], A What = [C W_{m+1}] G,
        // (M^H G) t = theta (What^H What) t with What^H What from the dots
        Mat Ah, Bh;
        if (prm.ritz_vectors) {
            Ah = dense::matmul(dense::adjoint(M), G);
            Bh = Mat(cols, cols);
            for (int i = 0; i < ke; ++i)
                for (int j = 0; j < ke; ++j) Bh(i, j) = d[i] * Dm(i, j) * d[j];
            for (int i = 0; i < mp; ++i)
                for (int j = 0; j < ke; ++j) {
                    Bh(ke + i, j) = M(ke + i, j);
                    Bh(j, ke + i) = std::conj(M(ke + i, j));
                }
            for (int i = 0; i < mp; ++i) Bh(ke + i, ke + i) = 1.0;
        }
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (prm.ritz_vectors)
                gen_ritz(Ah, Bh, kt, theta, sel, vecs, attempt == 1);
            else
                gen_harmonic(gf, M, &unorm, kt, theta, sel, vecs, attempt == 1);
            ritz_basis(sel, vecs, Pm);
            dense::qr_pos(dense::matmul(G, Pm), Qg, rg);
            if (well_conditioned_r(rg)) break;
        }
        const int kn = Pm.c;
        if (kn > KP) throw Fail{BGCR_ERR_NUMERICAL};
        const Mat PR = dense::matmul(Pm, dense::tri_inv_upper(rg));
        // inputs [U blocks, C blocks, V_1..V_meff, last]; outputs [U' blocks, C' blocks]
        const int nin = 2 * KB + me + 1;
        Mat K2(nin * P, 2 * KP);
        for (int c = 0; c < kn; ++c) {
            for (int i = 0; i < ke; ++i) {
                K2(i, c) = d[i] * PR(i, c);          // U D part of [U D  W_m] P rho^{-1}
                K2(KP + i, KP + c) = Qg(i, c);       // C part of [C W_{m+1}] Q
            }
            for (int i = 0; i < mp; ++i) {
                K2(2 * KP + i, c) = PR(ke + i, c);
                K2(2 * KP + i, KP + c) = Qg(ke + i, c);
            }
        }
        Mat lastQ = dense::matmul(co.RinvLast, Qg.block(ke + mp, 0, P, kn));
        for (int i = 0; i < P; ++i)
            for (int c = 0; c < kn; ++c) K2(2 * KP + mp + i, KP + c) = lastQ(i, c);
        std::vector<void*> out;
        const int o = 1 - cur;
        for (int b = 0; b < KB; ++b) out.push_back(ublk(o, b));
        for (int b = 0; b < KB; ++b) out.push_back(cblk(o, b));
        rp.active = true;
        rp.in = Q;
        rp.out = out;
        rp.K = K2;
        rp.kn = kn;
        rp.next_cur = o;
    }

    // End of a cycle (Algorithm 1): X += [V_m U] [Y; -F Y], R -= V_{m+1} H Y
    // (the recurrence; skipped in the precision form, whose outer loop takes
    // the FP64 true residual) and the refresh of (U, C).  The update and the
    // true residual (`residual_enqueue`, given by the caller) are queued
    // before the host solves the refresh problem, so the GPU computes them
    // meanwhile; the refresh combination follows.
    template <class FN>
    void finish_cycle(const CycleOut& co, bool withC, bool update_R, FN&& residual_enqueue) {
        update_solution(co, withC, update_R);
        residual_enqueue();
        RefreshPlan rp;
        if (k > 0) {
            if (withC)
                refresh_aug(co, rp);
            else
                refresh_first(co, rp);
        }
        if (rp.active) apply_refresh(rp);
    }

    int solve(const bgcr_csr* Am, const void* Bv, int64_t ldb, void* Xv, int64_t ldx, double tol,
              bgcr_stats* stt) override {
        const auto t0 = std::chrono::steady_clock::now();
        n_spmm = n_steps = n_cycles = n_refine = 0;
        alg_bytes = 0.0;
        n_deflated = 0;
        ilu_used = false;
        log_steps.clear();
        log_res.clear();
        int status = BGCR_OK;
        double rel = 0.0, relmax = 0.0;
        try {
            if (!Am || !Bv || !Xv || Am->n != n || !Am->row_ptr || !Am->col_idx || !Am->values || ldb < pu ||
                ldx < pu || !(tol > 0.0) || Am->nnz < 0 || Am->nnz > INT32_MAX)
                throw Fail{BGCR_ERR_INVALID};
            const A* B = (const A*)Bv;
            A* Xu = (A*)Xv;
            if (P > pu) {
                // enlarged block: B and X padded with zero columns to the block size
                HIPCHK(copy_block<A, A>(st, n, pu, B, ldb, Bpad, P, P));
                B = Bpad;
                ldb = P;
            }
            const T* avT = (const T*)Am->values;
            if (mixed) {
                if ((size_t)Am->nnz > av32_cap) {
                    if (av32) {
                        sync();
                        (void)hipFree(av32);
                        allocs.erase(std::find(allocs.begin(), allocs.end(), (void*)av32));
                    }
                    av32 = dalloc<float>((size_t)Am->nnz);
                    av32_cap = (size_t)Am->nnz;
                }
                HIPCHK(cast_values(st, (const double*)Am->values, av32, Am->nnz));
                avT = (const T*)av32;
            }
            HIPCHK(copy_block<A, A>(st, n, pu, Xu, ldx, X, P, P));
            std::vector<double> rn2, bn2;
            residual_norms(Am, B, ldb, R, rn2, bn2);
            double bn = 0.0, rn = 0.0;
            for (int b = 0; b < P; ++b) {
                bn += bn2[b];
                rn += rn2[b];
            }
            if (!std::isfinite(bn) || !std::isfinite(rn)) throw Fail{BGCR_ERR_NONFINITE};
            bn = std::sqrt(bn);
            rn = std::sqrt(rn);
            auto finish_norms = [&](const std::vector<double>& r2, const std::vector<double>& b2) {
                double s = 0.0;
                relmax = 0.0;
                for (int b = 0; b < P; ++b) {
                    s += r2[b];
                    if (b2[b] > 0.0) relmax = std::max(relmax, std::sqrt(r2[b] / b2[b]));
                }
                rel = bn > 0.0 ? std::sqrt(s) / bn : 0.0;
            };
            if (bn == 0.0) {
                HIPCHK(hipMemsetAsync(X, 0, (size_t)n * P * sizeof(A), st));
                rel = relmax = 0.0;
            } else {
                const double thresh = tol * bn;
                finish_norms(rn2, bn2);
                if (rn > thresh) {
                    if (pc) ilu_setup(Am);
                    if (!mixed)
                        status = run_plain(Am, avT, B, ldb, thresh, rn2, bn2, finish_norms);
                    else
                        status = run_mixed(Am, avT, B, ldb, thresh, rn2, bn2, finish_norms);
                }
            }
            HIPCHK(copy_block<A, A>(st, n, pu, X, P, Xu, ldx, pu));
            sync();
            if (!std::isfinite(rel)) status = BGCR_ERR_NONFINITE;
            if (ilu_used && ilu_wait_expired()) status = BGCR_ERR_NUMERICAL;
            // converged, with a rank-deficient block handled on the way
            if (status == BGCR_OK && n_deflated > 0) status = BGCR_BREAKDOWN_DEFLATED;
        } catch (const Fail& f) {
            status = f.code;
            (void)hipStreamSynchronize(st);
            hoff = 0;
        }
        if (stt) {
            std::memset(stt, 0, sizeof(*stt));
            stt->status = status;
            stt->cycles = n_cycles;
            stt->block_steps = n_steps;
            stt->spmm_calls = n_spmm;
            stt->rel_res = rel;
            stt->rel_res_max_col = relmax;
            stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            stt->alg_bytes = alg_bytes;
            stt->k_eff = keff;
            stt->refine_steps = n_refine;
            stt->deflations = n_deflated;
        }
        return status;
    }

    template <class FN>
    int run_plain(const bgcr_csr* Am, const T* avT, const A* B, int64_t ldb, double thresh,
                  std::vector<double>& rn2, std::vector<double>& bn2, FN& finish_norms) {
        bool pending = false;  // the last cycle's true residual is still to be logged
        bool queued = false;    // that residual is already queued (finish_cycle)
        bool prologued = false; // so is the next cycle's prologue
        auto enqueue = [&] {
            residual_enqueue(Am, B, ldb, nullptr);
            queued = true;
            // the prologue writes the start block into W2, which off the PIP
            // order may still hold V_{m+1} for the refresh, and an enlarged
            // start block is projected against the refreshed C: there it waits
            if (pip_order && P == pu) {
                cycle_prologue(false);  // wasted once per system, on the converged cycle
                prologued = true;
            }
        };
        if (keff > 0) {
            import_basis(Am, avT);
            project();
        } else {
            CycleOut co = cycle(Am, avT, false, thresh);
            finish_cycle(co, false, true, enqueue);
            ++n_cycles;
            log_steps.push_back(co.meff);
            log_res.push_back(0.0);
            pending = true;
        }
        for (;;) {
            const bool prologue_done = prologued;
            if (queued)
                residual_collect(rn2, bn2);
            else
                residual_norms(Am, B, ldb, nullptr, rn2, bn2);
            queued = prologued = false;
            double s = 0.0;
            for (double v : rn2) s += v;
            if (!std::isfinite(s)) throw Fail{BGCR_ERR_NONFINITE};
            finish_norms(rn2, bn2);
            if (pending) log_res.back() = rel_now(rn2, bn2);
            pending = false;
            if (std::sqrt(s) <= thresh) return BGCR_OK;
            if (n_cycles >= prm.max_cycles) return BGCR_NOT_CONVERGED;
            const bool withC = keff > 0;
            CycleOut co = cycle(Am, avT, withC, thresh, prologue_done);
            finish_cycle(co, withC, true, enqueue);
            ++n_cycles;
            log_steps.push_back(co.meff);
            log_res.push_back(0.0);
            pending = true;
        }
    }

    static double rel_now(const std::vector<double>& r2, const std::vector<double>& b2) {
        double a = 0.0, c = 0.0;
        for (size_t i = 0; i < r2.size(); ++i) {
            a += r2[i];
            c += b2[i];
        }
        return c > 0.0 ? std::sqrt(a / c) : 0.0;
    }

    template <class FN>
    int run_mixed(const bgcr_csr* Am, const T* avT, const A* B, int64_t ldb, double thresh,
                  std::vector<double>& rn2, std::vector<double>& bn2, FN& finish_norms) {
        if (keff > 0) import_basis(Am, avT);
        bool first = true;
        auto enqueue = [&] { residual_enqueue(Am, B, ldb, R); };
        for (;;) {
            if (!first) {
                residual_collect(rn2, bn2);  // queued by finish_cycle
                finish_norms(rn2, bn2);
                if (!log_steps.empty()) log_res.back() = rel_now(rn2, bn2);
            }
            first = false;
            double s = 0.0;
            for (double v : rn2) s += v;
            if (!std::isfinite(s)) throw Fail{BGCR_ERR_NONFINITE};
            if (std::sqrt(s) <= thresh) return BGCR_OK;
            if (n_cycles >= prm.max_cycles) return BGCR_NOT_CONVERGED;
            const bool withC = keff > 0;
            if (withC) project();
            CycleOut co = cycle(Am, avT, withC, thresh);
            finish_cycle(co, withC, false, enqueue);
            ++n_cycles;
            ++n_refine;
            log_steps.push_back(co.meff);
            log_res.push_back(0.0);
        }
    }

    int recycle_dim() const override { return keff; }

    void set_cycle_limit(int cycles) override { prm.max_cycles = std::max(1, cycles); }

    void get_profile(double* ms, double* bytes, int64_t* launches, int nclass) const override {
        for (int c = 0; c < nclass && c < BGCR_K_NCLASS; ++c) {
            if (ms) ms[c] = pms[c];
            if (bytes) bytes[c] = pby[c];
            if (launches) launches[c] = pcnt[c];
        }
    }

    int get_recycle(void* Uo, void* Co, int64_t ld) const override {
        if (ld < std::max(1, keff)) return BGCR_ERR_INVALID;
        auto* self = const_cast<Seq*>(this);
        try {
            for (int b = 0; b < KB; ++b) {
                const int cols = std::min(P, keff - b * P);
                if (cols <= 0) break;
                if (Uo)
                    HIPCHK(copy_block<TB, A>(self->st, n, cols, self->ublk(cur, b), P, (A*)Uo + (size_t)b * P, ld,
                                             cols));
                if (Co)
                    HIPCHK(copy_block<TB, A>(self->st, n, cols, self->cblk(cur, b), P, (A*)Co + (size_t)b * P, ld,
                                             cols));
            }
            self->sync();
        } catch (const Fail& f) {
            return f.code;
        }
        return BGCR_OK;
    }

    int set_recycle(const void* Ui, int64_t ld, int k_in) override {
        if (!Ui || k_in < 1 || k_in > KP || ld < k_in) return BGCR_ERR_INVALID;
        try {
            for (int b = 0; b < KB; ++b) {
                const int cols = std::max(0, std::min(P, k_in - b * P));
                if (cols > 0)
                    HIPCHK(copy_block<A, TB>(st, n, cols, (const A*)Ui + (size_t)b * P, ld, ublk(cur, b), P, P));
                else
                    HIPCHK(hipMemsetAsync(ublk(cur, b), 0, (size_t)n * P * sizeof(TB), st));
            }
            sync();
            keff = k_in;
        } catch (const Fail& f) {
            return f.code;
        }
        return BGCR_OK;
    }
};

// ---------------------------------------------------------------------------
// C ABI
namespace {

// ---------------------------------------------------------------------------
// Hybrid of Section 4.1.3 (p = 1): the first `budget` restart cycles of the
// sequence run on an enlarged-block sequence (block size L), every later
// cycle on a non-block one (L = 1); both share the caller's stream.  The
// switch happens at a restart: the enlarged sequence stops at its cycle
// limit, X holds its iterate, and the recycled U is handed over (as FP64
// columns) and imported by the L = 1 sequence at the start of its solve
// (A U = C S, T = C^H R), which is the identity up to rounding because the
// refreshed C satisfies C = A U, C^H C = I and C^H R = 0.
// ---------------------------------------------------------------------------
struct Hybrid final : bgcr_sequence {
    bgcr_sequence* big = nullptr;  // block size L
    bgcr_sequence* one = nullptr;  // block size 1
    int budget = 0;                // enlarged cycles left in the sequence
    int max_cycles = 1;
    bool moved = false;            // the recycled space lives in `one`
    void* ubuf = nullptr;          // n x ldu FP64 (complex128) columns of U
    int64_t ldu = 0;

    ~Hybrid() override {
        delete big;
        delete one;
        if (ubuf) (void)hipFree(ubuf);
    }
    bgcr_sequence* holder() const { return moved ? one : big; }

    int hand_over() {
        moved = true;
        const int ke = big->recycle_dim();
        if (ke <= 0) return BGCR_OK;
        const int rc = big->get_recycle(ubuf, nullptr, ldu);
        return rc != BGCR_OK ? rc : one->set_recycle(ubuf, ldu, ke);
    }

    int solve(const bgcr_csr* Am, const void* B, int64_t ldb, void* X, int64_t ldx, double tol,
              bgcr_stats* stt) override {
        const auto t0 = std::chrono::steady_clock::now();
        log_steps.clear();
        log_res.clear();
        bgcr_stats s1, s2;
        std::memset(&s1, 0, sizeof(s1));
        std::memset(&s2, 0, sizeof(s2));
        int status = BGCR_OK;
        bool second = false;
        auto take_log = [&](const bgcr_sequence* q) {
            log_steps.insert(log_steps.end(), q->log_steps.begin(), q->log_steps.end());
            log_res.insert(log_res.end(), q->log_res.begin(), q->log_res.end());
        };
        bool done = false;
        if (budget > 0) {
            big->set_cycle_limit(std::min(max_cycles, budget));
            status = big->solve(Am, B, ldb, X, ldx, tol, &s1);
            take_log(big);
            budget -= s1.cycles;
            // only a stop at the enlarged cycle limit continues with L = 1
            done = status != BGCR_NOT_CONVERGED || s1.cycles >= max_cycles || budget > 0;
            if (status == BGCR_BREAKDOWN_DEFLATED) status = BGCR_OK;
        }
        if (!done) {
            if (!moved) status = hand_over();
            if (status == BGCR_OK || status == BGCR_NOT_CONVERGED) {
                one->set_cycle_limit(max_cycles - s1.cycles);
                status = one->solve(Am, B, ldb, X, ldx, tol, &s2);
                take_log(one);
                second = true;
                if (status == BGCR_BREAKDOWN_DEFLATED) status = BGCR_OK;
            }
        }
        if (status == BGCR_OK && s1.deflations + s2.deflations > 0) status = BGCR_BREAKDOWN_DEFLATED;
        if (stt) {
            *stt = second ? s2 : s1;
            stt->status = status;
            stt->cycles = s1.cycles + s2.cycles;
            stt->block_steps = s1.block_steps + s2.block_steps;
            stt->spmm_calls = s1.spmm_calls + s2.spmm_calls;
            stt->alg_bytes = s1.alg_bytes + s2.alg_bytes;
            stt->refine_steps = s1.refine_steps + s2.refine_steps;
            stt->deflations = s1.deflations + s2.deflations;
            stt->k_eff = holder()->recycle_dim();
            stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return status;
    }
    int get_recycle(void* U, void* C, int64_t ld) const override { return holder()->get_recycle(U, C, ld); }
    int set_recycle(const void* U, int64_t ld, int k_in) override { return holder()->set_recycle(U, ld, k_in); }
    int recycle_dim() const override { return holder()->recycle_dim(); }
    void set_profiling(int on) override {
        big->set_profiling(on);
        one->set_profiling(on);
    }
    void get_profile(double* ms, double* bytes, int64_t* launches, int nclass) const override {
        const int nc = std::max(0, std::min(nclass, (int)BGCR_K_NCLASS));
        double m1[BGCR_K_NCLASS] = {}, b1[BGCR_K_NCLASS] = {}, m2[BGCR_K_NCLASS] = {}, b2[BGCR_K_NCLASS] = {};
        int64_t l1[BGCR_K_NCLASS] = {}, l2[BGCR_K_NCLASS] = {};
        big->get_profile(m1, b1, l1, nc);
        one->get_profile(m2, b2, l2, nc);
        for (int c = 0; c < nc; ++c) {
            if (ms) ms[c] = m1[c] + m2[c];
            if (bytes) bytes[c] = b1[c] + b2[c];
            if (launches) launches[c] = l1[c] + l2[c];
        }
    }
    void set_cycle_limit(int cycles) override { max_cycles = std::max(1, cycles); }
};

// the two halves of a hybrid: enlarged block without a switch, and L = 1
void hybrid_parts(const bgcr_params* prm, bgcr_params& big, bgcr_params& one) {
    big = *prm;
    big.enlarge_cycles = 0;
    one = big;
    one.block_size = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace of bgcr_apply_projected_noalloc: one array per GPU, resident until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device, looked up once per
// device on the first call there.
static __device__ __align__(256) unsigned char scratch[BGCR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BGCR_ERR_HIP;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BGCR_ERR_HIP;
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return BGCR_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int bgcr_create_sequence(const bgcr_params* prm, int64_t n, void* hip_stream, bgcr_sequence** out) {
    if (!out) return BGCR_ERR_INVALID;
    *out = nullptr;
    if (!valid_params(prm, n)) return BGCR_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BGCR_ERR_HIP;
    bgcr_sequence* s = nullptr;
    if (prm->enlarge_cycles > 0) {
        bgcr_params pb, p1;
        hybrid_parts(prm, pb, p1);
        auto* h = new (std::nothrow) Hybrid();
        if (!h) return BGCR_ERR_NOMEM;
        h->budget = prm->enlarge_cycles;
        h->max_cycles = prm->max_cycles;
        h->ldu = std::max(1, sizes_of(&pb, n).KP);
        int rc = bgcr_create_sequence(&pb, n, hip_stream, &h->big);
        if (rc == BGCR_OK) rc = bgcr_create_sequence(&p1, n, hip_stream, &h->one);
        if (rc == BGCR_OK && hipMalloc(&h->ubuf, (size_t)n * h->ldu * (prm->dtype == BGCR_C128 ? 16 : 8)) != hipSuccess)
            rc = BGCR_ERR_NOMEM;
        if (rc != BGCR_OK) {
            delete h;
            return rc;
        }
        *out = h;
        return BGCR_OK;
    }
    try {
        hipStream_t st = (hipStream_t)hip_stream;
        if (prm->dtype == BGCR_C128) {
            auto* q = new Seq<zd>(prm, n, st);
            s = q;
            q->allocate();
        } else if (prm->precision == BGCR_MIXED_FP32) {
            auto* q = new Seq<float>(prm, n, st);
            s = q;
            q->allocate();
        } else if (prm->precision == BGCR_MIXED_FP32_BF16) {
            auto* q = new Seq<float, bf16>(prm, n, st);
            s = q;
            q->allocate();
        } else {
            auto* q = new Seq<double>(prm, n, st);
            s = q;
            q->allocate();
        }
    } catch (const Fail& f) {
        delete s;
        return f.code;
    } catch (...) {
        delete s;
        return BGCR_ERR_NOMEM;
    }
    *out = s;
    return BGCR_OK;
}

int bgcr_solve(bgcr_sequence* s, const bgcr_csr* A, const void* B, int64_t ldb, void* X, int64_t ldx, double tol,
               bgcr_stats* st) {
    if (!s) return BGCR_ERR_INVALID;
    try {
        return s->solve(A, B, ldb, X, ldx, tol, st);
    } catch (...) {
        return BGCR_ERR_NOMEM;
    }
}

int bgcr_release(bgcr_sequence* s) {
    delete s;
    return BGCR_OK;
}

size_t bgcr_footprint_bytes(const bgcr_params* prm, int64_t n, int64_t nnz) {
    if (!valid_params(prm, n) || nnz < 0) return 0;
    if (prm->enlarge_cycles > 0) {
        bgcr_params pb, p1;
        hybrid_parts(prm, pb, p1);
        const size_t ub = (size_t)n * std::max(1, sizes_of(&pb, n).KP) * (prm->dtype == BGCR_C128 ? 16 : 8);
        return bgcr_footprint_bytes(&pb, n, nnz) + bgcr_footprint_bytes(&p1, n, nnz) + ub;
    }
    const Sizes z = sizes_of(prm, n);
    size_t b = z.total_fixed;
    if (prm->precision != BGCR_PLAIN_FP64) b += (size_t)nnz * sizeof(float);
    // ILU(0): the factors (A's pattern), the analysed column indices, and the
    // two level orders (n rows each, every level padded to chunks of 256 / P
    // rows; the analysis grows them when a pattern has many small levels)
    if (prm->precond == BGCR_PRECOND_ILU0) b += (size_t)nnz * (z.sa + sizeof(int)) + 2 * sizeof(int) * (size_t)n;
    return b;
}

int bgcr_recycle_dim(const bgcr_sequence* s, int32_t* k_eff) {
    if (!s || !k_eff) return BGCR_ERR_INVALID;
    *k_eff = s->recycle_dim();
    return BGCR_OK;
}

int bgcr_get_recycle(const bgcr_sequence* s, void* U_out, void* C_out, int64_t ld) {
    if (!s) return BGCR_ERR_INVALID;
    return s->get_recycle(U_out, C_out, ld);
}

int bgcr_set_recycle(bgcr_sequence* s, const void* U_in, int64_t ld, int32_t k_in) {
    if (!s) return BGCR_ERR_INVALID;
    return s->set_recycle(U_in, ld, k_in);
}

int bgcr_get_cycle_log(const bgcr_sequence* s, int32_t* steps, double* rel_res, int32_t cap, int32_t* count) {
    if (!s || !count || cap < 0) return BGCR_ERR_INVALID;
    const int c = (int)s->log_steps.size();
    *count = c;
    for (int i = 0; i < std::min(c, (int)cap); ++i) {
        if (steps) steps[i] = s->log_steps[i];
        if (rel_res) rel_res[i] = s->log_res[i];
    }
    return BGCR_OK;
}

int bgcr_spmm(const bgcr_csr* A, int32_t dtype, int32_t p, const void* V, void* W, void* hip_stream) {
    if (!A || !V || !W || A->n <= 0 || A->nnz < 0 || A->nnz > INT32_MAX || !A->row_ptr || !A->col_idx ||
        !A->values)
        return BGCR_ERR_INVALID;
    if (!(p == 1 || p == 2 || p == 4 || p == 8 || p == 16)) return BGCR_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BGCR_ERR_HIP;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    // the block SpMM of the Arnoldi step (row-layout kernel, 16 bytes of a row per lane)
    if (dtype == BGCR_F64)
        e = Launch<double>::spmm_rinv(st, p, A->n, A->nnz, A->row_ptr, A->col_idx, (const double*)A->values,
                                      (const double*)V, nullptr, nullptr, (double*)W, nullptr);
    else if (dtype == BGCR_C128)
        e = Launch<zd>::spmm_rinv(st, p, A->n, A->nnz, A->row_ptr, A->col_idx, (const zd*)A->values, (const zd*)V,
                                  nullptr, nullptr, (zd*)W, nullptr);
    else
        return BGCR_ERR_INVALID;
    return e == hipSuccess ? BGCR_OK : BGCR_ERR_HIP;
}

// blocks of C per dot or update launch, and workgroups, of bgcr_apply_projected
static int proj_chunk(int p) { return p >= 8 ? 16 : 32; }
static constexpr int PROJ_NWG = 512;

size_t bgcr_apply_projected_work_bytes(int64_t n, int32_t p, int32_t kc) {
    if (!(p == 1 || p == 2 || p == 4 || p == 8 || p == 16) || kc < 0 || n < 0) return 0;
    const size_t ch = (size_t)std::max(1, std::min(kc, proj_chunk(p)));
    // S (kc p x p) and the partials of one launch (PROJ_NWG x chunk p x p; the
    // update sweeps also write a p x p Gram per workgroup)
    return sizeof(double) * ((size_t)std::max(kc, 1) * p * p + (size_t)PROJ_NWG * (ch + 1) * p * p);
}

static int apply_projected(const bgcr_csr* A, int32_t p, int32_t kc, const double* C, const double* V, double* W,
                           int32_t variant, void* work, size_t work_bytes, void* hip_stream) {
    if (!A || !V || !W || V == W || !work || A->n <= 0 || A->nnz < 0 || A->nnz > INT32_MAX || !A->row_ptr ||
        !A->col_idx || !A->values)
        return BGCR_ERR_INVALID;
    if (!(p == 1 || p == 2 || p == 4 || p == 8 || p == 16) || kc < 0 || (kc > 0 && !C) ||
        (variant != 0 && variant != 1))
        return BGCR_ERR_INVALID;
    if (work_bytes < bgcr_apply_projected_work_bytes(A->n, p, kc)) return BGCR_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BGCR_ERR_HIP;
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t n = A->n;
    const int P2 = p * p;
    double* S = (double*)work;
    double* part = S + (size_t)std::max(kc, 1) * P2;
    auto blocks = [&](int b0, int nb) {
        BlockPtrs q;
        std::memset(&q, 0, sizeof(q));
        for (int b = 0; b < nb; ++b) q.p[b] = C + (size_t)(b0 + b) * n * p;
        return q;
    };
    // S[b0 ..] = C_{b0 ..}^T W for nb blocks
    auto dots = [&](int b0, int nb) -> hipError_t {
        BlockPtrs w;
        std::memset(&w, 0, sizeof(w));
        w.p[0] = W;
        const hipError_t e = mfma_dot<double>(st, p, n, w, 1, blocks(b0, nb), nb, part, nullptr, PROJ_NWG);
        if (e != hipSuccess) return e;
        return reduce_partials<double>(st, part, PROJ_NWG, nb * P2, nullptr, S + (size_t)b0 * P2, nullptr);
    };
    // W -= C_{b0 ..} S[b0 ..] in place
    auto update = [&](int b0, int nb) -> hipError_t {
        const double* Sb = S + (size_t)b0 * P2;
        if (p == 1) return narrow_sweep<double>(st, n, W, blocks(b0, nb), nb, Sb, W, part, PROJ_NWG, nullptr, false);
        if (p == 2)
            return Launch<double>::update_dot(st, p, n, W, blocks(b0, nb), nb, Sb, nullptr, W, 0, 1, part, PROJ_NWG,
                                              nullptr, 2);
        return mfma_proj_gram<double>(st, p, n, W, blocks(b0, nb), nb, Sb, W, part, nullptr, PROJ_NWG);
    };
    hipError_t e = Launch<double>::spmm_rinv(st, p, n, A->nnz, A->row_ptr, A->col_idx, (const double*)A->values, V,
                                              nullptr, nullptr, W, nullptr);
    const int ch = proj_chunk(p);
    if (variant == 0) {
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            for (int b0 = 0; b0 < kc && e == hipSuccess; b0 += ch) e = dots(b0, std::min(ch, kc - b0));
            for (int b0 = 0; b0 < kc && e == hipSuccess; b0 += ch) e = update(b0, std::min(ch, kc - b0));
        }
    } else {
        for (int b = 0; b < kc && e == hipSuccess; ++b) {
            e = dots(b, 1);
            if (e == hipSuccess) e = update(b, 1);
        }
    }
    return e == hipSuccess ? BGCR_OK : BGCR_ERR_HIP;
}

int bgcr_apply_projected(const bgcr_csr* A, int32_t p, int32_t kc, const double* C, const double* V, double* W,
                         int32_t variant, void* work, size_t work_bytes, void* hip_stream) {
    return apply_projected(A, p, kc, C, V, W, variant, work, work_bytes, hip_stream);
}

int bgcr_apply_projected_noalloc(const bgcr_csr* A, int32_t p, int32_t kc, const double* C, const double* V,
                                 double* W, int32_t variant, void* hip_stream) {
    if (!A || A->n <= 0) return BGCR_ERR_INVALID;
    const size_t need = bgcr_apply_projected_work_bytes(A->n, p, kc);
    if (need == 0 || need > (size_t)BGCR_NOALLOC_SCRATCH_BYTES) return BGCR_ERR_INVALID;
    void* ptr = nullptr;
    const int rc = noalloc_scratch(&ptr);
    if (rc != BGCR_OK) return rc;
    return apply_projected(A, p, kc, C, V, W, variant, ptr, (size_t)BGCR_NOALLOC_SCRATCH_BYTES, hip_stream);
}

int bgcr_set_profiling(bgcr_sequence* s, int on) {
    if (!s) return BGCR_ERR_INVALID;
    try {
        s->set_profiling(on);
    } catch (...) {
        return BGCR_ERR_HIP;
    }
    return BGCR_OK;
}

int bgcr_get_profile(const bgcr_sequence* s, double* ms, double* bytes, int64_t* launches, int32_t nclass) {
    if (!s || nclass < 0) return BGCR_ERR_INVALID;
    s->get_profile(ms, bytes, launches, nclass);
    return BGCR_OK;
}

const char* bgcr_strerror(int status) {
    switch (status) {
        case BGCR_OK: return "ok";
        case BGCR_NOT_CONVERGED: return "not converged within max_cycles";
        case BGCR_BREAKDOWN_DEFLATED: return "converged; a rank-deficient block was handled on the way";
        case BGCR_ERR_INVALID: return "invalid argument";
        case BGCR_ERR_NOMEM: return "device out of memory";
        case BGCR_ERR_HIP: return "HIP runtime error";
        case BGCR_ERR_NONFINITE: return "non-finite value";
        case BGCR_ERR_NUMERICAL: return "numerical failure (rank-deficient block or eigensolver)";
        default: return "unknown status";
    }
}

}  // extern "C"
