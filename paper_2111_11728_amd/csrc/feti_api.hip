// C ABI of the FETI library: context, setup pipeline, Krylov drivers, recovery.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "feti.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace feti;

namespace {

thread_local std::string g_err;

feti_status fail(feti_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

struct HipError {
    std::string msg;
};

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) throw HipError{std::string(#x) + ": " + hipGetErrorString(e_)};      \
    } while (0)

#define CHECK_LAUNCH() HIPCHK(hipGetLastError())

// Workspace of feti_apply_F_noalloc: the local products Y_s, the corner rows T_s and the coarse
// vectors t and v of one F*Lambda. Every GPU the library runs on holds its own copy until the
// process ends; calls on one GPU share it, so such calls must not overlap in time.
constexpr long long kNoAllocScratchBytes = 16LL << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of this GPU's copy of scratch, looked up once per device with that device
// current (host code never passes the array's name itself to a kernel or a copy).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw HipError{"device ordinal out of range for the no-allocation workspace"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Unit-modulus element stiffness by full Gauss quadrature on the unit square / cube
// (bilinear / trilinear shape functions, corners x fastest, DOFs interleaved).
std::vector<double> element_K0(int dim, double nu) {
    const int nc = 1 << dim, ne = dim * nc, ns = dim == 2 ? 3 : 6;
    std::vector<double> D(ns * ns, 0.0), K(ne * ne, 0.0);
    if (dim == 2) {
        const double c = 1.0 / (1.0 - nu * nu);
        D[0] = c; D[1] = c * nu; D[3] = c * nu; D[4] = c; D[8] = c * 0.5 * (1.0 - nu);
    } else {
        const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = 1.0 / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[i * 6 + j] = lam + (i == j ? 2.0 * mu : 0.0);
        for (int i = 3; i < 6; ++i) D[i * 6 + i] = mu;
    }
    const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    const int ngp = 1 << dim;
    std::vector<double> B(ns * ne);
    for (int g = 0; g < ngp; ++g) {
        const double xi[3] = {gp[g & 1], gp[(g >> 1) & 1], dim == 3 ? gp[(g >> 2) & 1] : 0.0};
        const double w = dim == 2 ? 0.25 : 0.125;
        std::fill(B.begin(), B.end(), 0.0);
        for (int a = 0; a < nc; ++a) {
            const int o[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
            double dN[3];
            for (int d = 0; d < dim; ++d) {
                double v = o[d] ? 1.0 : -1.0;
                for (int d2 = 0; d2 < dim; ++d2)
                    if (d2 != d) v *= o[d2] ? xi[d2] : 1.0 - xi[d2];
                dN[d] = v;
            }
            if (dim == 2) {
                B[0 * ne + 2 * a] = dN[0];
                B[1 * ne + 2 * a + 1] = dN[1];
                B[2 * ne + 2 * a] = dN[1];
                B[2 * ne + 2 * a + 1] = dN[0];
            } else {
                B[0 * ne + 3 * a] = dN[0];
                B[1 * ne + 3 * a + 1] = dN[1];
                B[2 * ne + 3 * a + 2] = dN[2];
                B[3 * ne + 3 * a + 1] = dN[2];
                B[3 * ne + 3 * a + 2] = dN[1];
                B[4 * ne + 3 * a] = dN[2];
                B[4 * ne + 3 * a + 2] = dN[0];
                B[5 * ne + 3 * a] = dN[1];
                B[5 * ne + 3 * a + 1] = dN[0];
            }
        }
        for (int i = 0; i < ne; ++i)
            for (int j = 0; j < ne; ++j) {
                double v = 0.0;
                for (int p = 0; p < ns; ++p)
                    for (int q = 0; q < ns; ++q) v += B[p * ne + i] * D[p * ns + q] * B[q * ne + j];
                K[i * ne + j] += w * v;
            }
    }
    return K;
}

long long rup(long long x, long long m) { return (x + m - 1) / m * m; }

// FETI_VERBOSE=1 prints one line per Krylov iteration (and per restart) to stderr.
int verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("FETI_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v;
}

}  // namespace

// -----------------------------------------------------------------------------------------
struct feti_ctx {
    Plan P;
    feti_opts opts{};
    double p = 3, E0 = 1, Emin = 1e-6;
    hipStream_t st = nullptr;
    DevTopo t;
    std::vector<SubMeta> hsubs;
    std::vector<LineMeta> hlines;
    std::vector<void*> allocs;
    long long bytes = 0;

    // numeric state
    double* Emod = nullptr;   // SIMP moduli of the elements, per setup (Sec. 1, Eq. 1)
    double *rho = nullptr, *L = nullptr, *Li = nullptr, *Z = nullptr, *S = nullptr, *diag = nullptr, *F64 = nullptr;
    double* sw64 = nullptr;
    float* sw32 = nullptr;
    __hip_bfloat16 *swhi = nullptr, *swlo = nullptr;
    double *Pk = nullptr, *W1 = nullptr, *W2 = nullptr, *ypart = nullptr;
    float* Pk32 = nullptr;   // opts.precond_fp32: the packed preconditioner tiles rounded to FP32
    long long n_Pk = 0;
    double *Kc = nullptr, *Kcc = nullptr, *Kcc_w = nullptr, *Kcc_inv = nullptr;
    // designs held by the context (one, or several independent ones as a disjoint union)
    std::vector<DesignMeta> designs;
    bool segmented = false;   // several designs, each with its own S-FETI directions
    // F*Lambda tile shapes (chosen by feti_autotune, defaults otherwise) and the per-subdomain
    // round-off verdicts of the hybrid lists
    feti_tuning tune{2 * kFlWaves, kFlWaves, 1, 4, 0.0, 0.0, 0};
    std::vector<int> sub_ok;
    // captured per-iteration sequences (opts.graphs): F*Lambda per precision, preconditioner
    struct GraphSlot {
        hipGraph_t g = nullptr;
        hipGraphExec_t e = nullptr;
        int key = -1;
    };
    GraphSlot g_apply[3], g_prec;
    void drop_graphs() {
        for (GraphSlot* gs : {&g_apply[0], &g_apply[1], &g_apply[2], &g_prec}) {
            if (gs->e) hipGraphExecDestroy(gs->e);
            if (gs->g) hipGraphDestroy(gs->g);
            *gs = GraphSlot{};
        }
    }
    // module types (opts.recycle): subdomains with the same local layout (structural key) and the
    // same densities share one setup; rep_of[s] is the subdomain whose operators s uses
    std::vector<unsigned long long> skey;
    std::vector<int> rep_of;
    std::vector<SubMeta> hsubs_act;   // what t.subs holds: operator offsets of each representative
    int n_setup_subs = 0;
    bool aliased = false;
    SubMeta* subs_dev = nullptr;      // t.subs, writable
    SubMeta* subs_rep = nullptr;      // representatives' own SubMeta, compacted
    GemmDesc *d_syrk_r = nullptr, *d_F_r = nullptr;
    PotrfDesc* d_potrf_r = nullptr;
    TrsmDesc* d_trsm_r = nullptr;
    std::vector<GemmDesc> h_dsy, h_dF;
    std::vector<PotrfDesc> h_dpo;
    std::vector<TrsmDesc> h_dtr;
    unsigned long long* hash_dev = nullptr;
    int *pair_dev = nullptr, *flag_dev = nullptr, *map_dev = nullptr;
    double* rbm_tmp = nullptr;        // compacted Total FETI per-subdomain results before expansion
    void* scratch = nullptr;   // this device's no-allocation workspace (scratch_address)
    bool have_lam = false;     // lam_prev holds the multipliers of the last solve (warm start)
    FlTile *fl64_dev = nullptr, *flred_dev = nullptr;
    int fl64_cap = 0, flred_cap = 0;
    std::vector<CoarseBlk> hcblk;
    GemmDesc* d_cc_gemm = nullptr;
    PotrfDesc* d_cc_potrf = nullptr;
    TrsmDesc* d_cc_trsm = nullptr;
    std::vector<double> eps0_d, true_d;   // per design: initial and last true preconditioned residual
    double *Rb = nullptr, *Cit = nullptr, *tau = nullptr, *GG = nullptr, *GG_w = nullptr, *GG_inv = nullptr;
    double *w = nullptr, *bg_w = nullptr;
    int* info = nullptr;
    char* bt_ws = nullptr;   // plane-by-plane band Cholesky: descriptors and pivot flags
    double* bt_T = nullptr;  // plane-by-plane L^{-1} K_i,beta: one plane block per subdomain
    GemmDesc *d_syrk = nullptr, *d_F = nullptr, *d_one = nullptr;
    PotrfDesc *d_potrf = nullptr, *d_potrf_one = nullptr;
    TrsmDesc *d_trsm = nullptr, *d_trsm_one = nullptr;
    int syrk_tdim = 0, F_tdim = 0, max_nb_cols = 0;
    int n_alpha = 0;
    // deflation of local interface modes (opts.defl_modes): local operators at off_P (F_s factor,
    // omega S~ omega, their product, C_s), interface weights omega, modes U (8 per interface DOF),
    // eigenvalues, counts and first columns per subdomain, the dual vectors Y and their
    // F-orthonormal blocks dfW / dfQ (n_lambda x 64 each, df_nd of them kept)
    double *dfL = nullptr, *dfM = nullptr, *dfB = nullptr, *dfC = nullptr, *dfOmega = nullptr, *dfU = nullptr,
           *dfMu = nullptr, *dfY = nullptr, *dfPsi = nullptr, *dfPad = nullptr;
    int *dfCnt = nullptr, *dfCol0 = nullptr;
    GemmDesc* d_df = nullptr;
    std::vector<double*> dfW, dfQ;
    const double** dfW_dev = nullptr;
    const double** dfQ_dev = nullptr;
    int df_cap = 0, df_nd = 0, n_defl = 0, n_defl_kept = 0;

    // solve buffers
    double *f_last = nullptr, *fi = nullptr, *fbeta = nullptr, *h = nullptr, *g = nullptr, *yb = nullptr,
           *yc = nullptr, *fbar_s = nullptr, *d = nullptr, *lam0 = nullptr, *lam = nullptr, *lt = nullptr,
           *lt2 = nullptr, *lam_prev = nullptr, *r = nullptr, *xb = nullptr, *ubeta = nullptr, *ui = nullptr, *uloc = nullptr, *uc = nullptr,
           *alpha = nullptr, *e = nullptr, *GY = nullptr, *tcoef = nullptr, *u_int = nullptr;
    double *Ybuf = nullptr, *Tbuf = nullptr, *vbuf = nullptr, *Qtmp = nullptr, *Tsum = nullptr;
    double *Zk = nullptr, *Qk = nullptr, *Delta = nullptr, *Tm = nullptr, *gam = nullptr, *part = nullptr,
           *scal = nullptr, *Psi = nullptr, *tmpv = nullptr, *zv = nullptr, *K0dev = nullptr;
    int* rank_dev = nullptr;         // inside scal (scal[8]), so one copy returns eps and rank
    double* hpin = nullptr;          // pinned host mirror of scal
    // one-ahead S-FETI loop: per-iteration copies of scal (two slots), published by the device
    double* hslot[2] = {nullptr, nullptr};       // coherent, host-mapped: scalars, then a sequence number
    double* hslot_dev[2] = {nullptr, nullptr};   // their device addresses
    long long pub_seq = 0;                       // last sequence number published
    const double** qk_ptr = nullptr;    // device table holding the single pointer Qk
    const double** zk_ptr = nullptr;    // device table holding the single pointer Zk
    double* tcbuf = nullptr;            // coarse right-hand sides t (n_cg x k)
    // per-subdomain precision selection for the reduced-precision F*Lambda (FETI-DP)
    double* pivdev = nullptr;
    // hybrid F*Lambda work lists: reduced rows where safe, and the FP64 rest (owned buffers)
    FlTile* fl_hyb_dev = nullptr;
    int fl_hyb_cap = 0;
    FlTiles fl_hyb;   // in-solve reduced-precision form: reduced tiles, then FP64 split-contraction tiles
    bool hybrid = false;
    int n_fp64_subs = 0;
    long long psi_cap = 0;
    // history of F-orthonormal directions
    std::vector<double*> hist_chunks;
    std::vector<const double*> WH, QH;
    const double** WH_dev = nullptr;
    const double** QH_dev = nullptr;
    int hist_cap = 0, hist_kd = 0;
    bool have_f = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double last_ms[4] = {0, 0, 0, 0};

    template <typename T>
    T* alloc(long long n) {
        if (n <= 0) n = 1;
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, sizeof(T) * n));
        allocs.push_back(p);
        bytes += sizeof(T) * n;
        return (T*)p;
    }
    template <typename T>
    T* upload(const std::vector<T>& v) {
        T* p = alloc<T>((long long)v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
        return p;
    }
    ~feti_ctx() {
        hipStreamSynchronize(st);
        drop_graphs();
        for (void* p : allocs) hipFree(p);
        for (double* p : hist_chunks) hipFree(p);
        if (hpin) hipHostFree(hpin);
        for (int q = 0; q < 2; ++q) {
            if (hslot[q]) hipHostFree(hslot[q]);
        }
        if (WH_dev) hipFree(WH_dev);
        if (QH_dev) hipFree(QH_dev);
        if (Psi) hipFree(Psi);
        if (fl_hyb_dev) hipFree(fl_hyb_dev);
        if (fl64_dev) hipFree(fl64_dev);
        if (flred_dev) hipFree(flred_dev);
        for (auto& e : ev)
            if (e) hipEventDestroy(e);
    }
};

namespace {

// Packs per-subdomain row-block ranges into F*Lambda tiles. Workgroup i runs on XCD i mod 8,
// so the tiles of one subdomain, which gather the same X_s, are kept in one XCD's bucket (one
// L2). A tile's time is taken as its contraction length ldF times the wavefronts its busiest
// SIMD runs; an XCD's 32 CUs take its tiles longest first, each tile going to the CU that
// frees first. Subdomains are placed largest first, each on the XCD whose finishing time so
// modelled grows least (ties: the least work), and every bucket lists its tiles longest
// first. Uneven buckets are padded with empty slots.
struct RbRange {
    int red0, n_red, d0, n_d;
};
// max_d caps the FP64 row blocks of one tile (small tiles spread FP64 work over many CUs);
// xcd = false lists the tiles in order (no XCD grouping, no empty slots).
std::vector<FlTile> pack_tiles(const std::vector<RbRange>& rr, const std::vector<int>& ld, int flags = 0,
                               int max_d = kFlWaves, bool xcd = true, int max_red = 2 * kFlWaves) {
    const int ns = (int)rr.size();
    std::vector<std::vector<FlTile>> per(ns);
    std::vector<double> cost(ns, 0.0);
    auto tile_cost = [&](const FlTile& T) {
        const int waves = (T.n_red + 1) / 2 + T.n_d;
        return (double)ld[T.s] * ((waves + 3) / 4);
    };
    for (int s = 0; s < ns; ++s) {
        RbRange r = rr[s];
        while (r.n_red > 0 || r.n_d > 0) {
            FlTile T{s, r.red0, std::min({r.n_red, 2 * kFlWaves, max_red}), r.d0, 0, flags, 0, 0};
            const int mixed = (flags & kFlSplitK) ? 0 : ((T.n_red & 1) && r.n_d > 0 ? 1 : 0);
            T.n_d = std::min({r.n_d, max_d, kFlWaves - (T.n_red + 1) / 2 + mixed});
            r.red0 += T.n_red;
            r.n_red -= T.n_red;
            r.d0 += T.n_d;
            r.n_d -= T.n_d;
            per[s].push_back(T);
            cost[s] += tile_cost(T);
        }
    }
    if (!xcd) {
        std::vector<FlTile> out;
        for (auto& v : per) out.insert(out.end(), v.begin(), v.end());
        return out;
    }
    std::vector<int> order(ns);
    for (int s = 0; s < ns; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    constexpr int kCuPerXcd = 32;
    std::vector<std::vector<FlTile>> bucket(8);
    std::vector<std::vector<double>> cu(8, std::vector<double>(kCuPerXcd, 0.0));   // min-heaps
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto place = [&](std::vector<double>& h, const std::vector<FlTile>& tiles) {
        double end = 0.0;
        for (const FlTile& T : tiles) {   // tiles of one subdomain: equal or decreasing cost
            std::pop_heap(h.begin(), h.end(), std::greater<double>());
            h.back() += tile_cost(T);
            end = std::max(end, h.back());
            std::push_heap(h.begin(), h.end(), std::greater<double>());
        }
        return end;
    };
    for (int s : order) {
        if (per[s].empty()) continue;
        std::sort(per[s].begin(), per[s].end(), [&](const FlTile& a, const FlTile& c) { return tile_cost(a) > tile_cost(c); });
        int best = 0;
        double best_end = 0.0;
        for (int x = 0; x < 8; ++x) {
            std::vector<double> h = cu[x];
            const double end = std::max(*std::max_element(h.begin(), h.end()), place(h, per[s]));
            if (x == 0 || end < best_end || (end == best_end && load[x] < load[best])) {
                best = x;
                best_end = end;
            }
        }
        place(cu[best], per[s]);
        load[best] += cost[s];
        bucket[best].insert(bucket[best].end(), per[s].begin(), per[s].end());
    }
    for (auto& b : bucket)
        std::stable_sort(b.begin(), b.end(), [&](const FlTile& a, const FlTile& c) { return tile_cost(a) > tile_cost(c); });
    size_t mx = 0;
    for (auto& b : bucket) mx = std::max(mx, b.size());
    std::vector<FlTile> out;
    for (size_t i = 0; i < mx; ++i)
        for (int x = 0; x < 8; ++x)
            out.push_back(i < bucket[x].size() ? bucket[x][i] : FlTile{-1, 0, 0, 0, 0, 0, 0, 0});
    while (!out.empty() && out.back().s < 0) out.pop_back();
    return out;
}

// F*Lambda work lists for the context's tile shapes (c->tune): every row block in FP64, every
// row block in the reduced precision, and, after the round-off test, the hybrid lists:
// subdomains that passed get reduced precision for their F_s row blocks and FP64 for the blocks
// holding F_rc^T rows (the coarse right-hand side stays FP64: Kbar_cc^{-1} amplifies its errors)
// in the same tile; subdomains that failed run in FP64, in a second launch of split-contraction
// tiles spread over many CUs.
void build_fl_tiles(feti_ctx* c) {
    c->drop_graphs();   // captured launches refer to the old tile lists
    DevTopo& t = c->t;
    const int ns = c->P.n_sub;
    const feti_tuning& q = c->tune;
    auto put = [&](const std::vector<FlTile>& v, FlTile*& dev, int& cap, FlTiles& out) {
        if ((int)v.size() > cap) {
            if (dev) {
                HIPCHK(hipStreamSynchronize(c->st));
                HIPCHK(hipFree(dev));
            }
            HIPCHK(hipMalloc(&dev, sizeof(FlTile) * std::max<size_t>(1, v.size())));
            cap = (int)v.size();
        }
        if (!v.empty()) HIPCHK(hipMemcpyAsync(dev, v.data(), sizeof(FlTile) * v.size(), hipMemcpyHostToDevice, c->st));
        out = FlTiles{dev, (int)v.size()};
    };
    std::vector<RbRange> r64(ns), rred(ns);
    std::vector<int> ld(ns);
    for (int s = 0; s < ns; ++s) {
        ld[s] = c->hsubs[s].ldF;
        const int nrb = c->hsubs[s].rows_F / 16;
        r64[s] = RbRange{0, 0, 0, nrb};
        rred[s] = RbRange{0, nrb, 0, 0};
    }
    put(pack_tiles(r64, ld, 0, q.max_d, q.xcd != 0), c->fl64_dev, c->fl64_cap, t.fl64);
    put(pack_tiles(rred, ld, 0, q.max_d, q.xcd != 0, q.max_red), c->flred_dev, c->flred_cap, t.flred);
    if (c->hybrid && (int)c->sub_ok.size() == ns) {
        std::vector<RbRange> rr(ns), rd(ns);
        for (int s = 0; s < ns; ++s) {
            const SubMeta& M = c->hsubs[s];
            const int nrb = M.rows_F / 16, t0 = M.n_c > 0 ? M.rowT / 16 : nrb;
            rr[s] = c->sub_ok[s] ? RbRange{0, t0, t0, nrb - t0} : RbRange{0, 0, 0, 0};
            rd[s] = c->sub_ok[s] ? RbRange{0, 0, 0, 0} : RbRange{0, 0, 0, nrb};
        }
        // one launch: the FP64 split-contraction tiles follow the reduced ones and fill the CUs
        // those leave free (the kernel dispatches a tile by its flags, whatever the precision)
        // (split_d = 0: the failed subdomains as plain FP64 tiles of up to max_d row blocks, one per
        // wavefront; fp64_first: their tiles lead the launch instead of following it)
        std::vector<FlTile> hyb = pack_tiles(rr, ld, kFlNoT, q.max_d, q.xcd != 0, q.max_red);
        const std::vector<FlTile> h64 =
            q.split_d > 0 ? pack_tiles(rd, ld, kFlSplitK, q.split_d, false) : pack_tiles(rd, ld, 0, q.max_d, false);
        if (q.fp64_first)
            hyb.insert(hyb.begin(), h64.begin(), h64.end());
        else
            hyb.insert(hyb.end(), h64.begin(), h64.end());
        put(hyb, c->fl_hyb_dev, c->fl_hyb_cap, c->fl_hyb);
    }
    HIPCHK(hipStreamSynchronize(c->st));
}

void build_layout(feti_ctx* c) {
    Plan& P = c->P;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    c->scratch = scratch_address(dev);
    const int ns = P.n_sub;
    if (c->designs.empty()) {   // a single design: the whole plan
        DesignMeta D;
        D.n_sub = ns;
        D.n_el = P.n_el;
        D.n_nodes = P.n_nodes;
        D.n_dof = P.n_dof;
        D.n_lambda = P.n_lambda;
        D.n_rows = P.n_lambda;
        D.n_cg = P.n_cg;
        D.n_groups = P.n_groups;
        for (int a = 0; a < 3; ++a) {
            D.nel[a] = P.nel[a];
            D.nsub[a] = P.nsub[a];
            D.ax_first[a] = P.ax_first[a];
            D.ax_cnt[a] = P.ax_cnt[a];
        }
        c->designs.push_back(D);
    }
    std::vector<int> sub_design(ns, 0);
    for (int d = 0; d < (int)c->designs.size(); ++d)
        for (int s = 0; s < c->designs[d].n_sub; ++s) sub_design[c->designs[d].sub0 + s] = d;
    c->hsubs.assign(ns, SubMeta{});
    c->hlines.clear();
    long long oL = 0, oZ = 0, oS = 0, oF = 0, oP = 0, oPk = 0, oKc = 0, oR = 0, oLi = 0;
    DevTopo& t = c->t;
    const int nrbm = P.method == FETI_TFETI ? (P.dim == 2 ? 3 : 6) : 0;
    for (int s = 0; s < ns; ++s) {
        SubMeta& M = c->hsubs[s];
        for (int a = 0; a < 3; ++a) {
            M.lo[a] = P.lo[3 * s + a];
            M.nn[a] = P.nn[3 * s + a];
        }
        {
            const DesignMeta& D = c->designs[sub_design[s]];
            M.nelx = D.nel[0];
            M.nely = D.nel[1];
            M.el0 = D.el0;
        }
        M.n_loc = P.n_loc[s];
        M.n_i = P.n_i[s];
        M.n_b = P.n_b[s];
        M.n_c = P.n_c[s];
        M.n_beta = M.n_b + M.n_c;
        M.grp = P.grp[s];
        M.ldF = (int)rup(std::max(M.n_b, 1), 32);
        M.rowT = M.n_b;
        M.rows_F = (int)rup(std::max(M.n_b + M.n_c, 1), 16);
        M.off_loc = P.off_loc[s];
        M.off_i = P.off_i[s];
        M.off_b = P.off_b[s];
        M.off_c = P.off_c[s];
        // lines: grid rows (2D) or planes (3D) of interior DOFs
        const int nlines = P.dim == 2 ? M.nn[1] : M.nn[2];
        const int per_line_nodes = P.dim == 2 ? M.nn[0] : M.nn[0] * M.nn[1];
        M.n_lines = nlines;
        t.max_planes = std::max(t.max_planes, nlines);
        M.line0 = (long long)c->hlines.size();
        M.off_L = oL;
        int i0 = 0, prev = 0;
        for (int k = 0; k < nlines; ++k) {
            int n = 0;
            for (int ln = k * per_line_nodes; ln < (k + 1) * per_line_nodes; ++ln)
                for (int cc = 0; cc < P.dim; ++cc)
                    if (P.lcls[M.off_loc + (long long)ln * P.dim + cc] == CLS_I) ++n;
            LineMeta Lm{};
            Lm.i0 = i0;
            Lm.n = n;
            Lm.n_prev = prev;
            Lm.off_diag = oL;
            oL += (long long)n * n;
            Lm.off_sub = oL;
            oL += (long long)n * prev;
            Lm.off_inv = oLi;
            oLi += (long long)n * n;
            c->hlines.push_back(Lm);
            t.max_line = std::max(t.max_line, n);
            i0 += n;
            prev = n;
        }
        M.off_Z = oZ;
        oZ += (long long)M.n_i * M.n_beta;
        M.off_S = oS;
        oS += (long long)M.n_beta * M.n_beta;
        M.off_F = oF;
        M.off_Fsw = oF;
        oF += (long long)M.rows_F * M.ldF;
        M.off_P = oP;
        oP += (long long)M.n_b * M.n_b;
        M.off_Pk = oPk;
        oPk += (long long)((M.n_b + 63) / 64) * ((M.n_b + 63) / 64 + 1) / 2 * 4096;
        M.off_Kc = oKc;
        oKc += (long long)M.n_c * M.n_c;
        M.off_R = oR;
        oR += (long long)M.n_b * nrbm;
        t.max_nodes = std::max(t.max_nodes, M.nn[0] * M.nn[1] * M.nn[2]);
        t.max_beta = std::max(t.max_beta, M.n_beta);
        t.max_nb = std::max(t.max_nb, M.n_b);
        t.max_nc = std::max(t.max_nc, M.n_c);
        t.max_ni = std::max(t.max_ni, M.n_i);
        t.max_nloc = std::max(t.max_nloc, M.n_loc);
        t.max_rows_F = std::max(t.max_rows_F, M.rows_F);
    }
    t.dim = P.dim;
    t.n_sub = ns;
    t.n_lines_tot = (int)c->hlines.size();
    t.n_lambda = P.n_lambda;
    t.n_cg = P.n_cg;
    t.n_groups = P.n_groups;
    t.n_rbm = nrbm;
    for (int a = 0; a < 3; ++a) {
        t.nel[a] = P.dim > a ? P.nel[a] : 0;
        t.nsub[a] = P.nsub[a];
    }
    t.nb_tot = P.off_b[ns];
    t.nc_tot = P.off_c[ns];
    t.ni_tot = P.off_i[ns];
    t.nloc_tot = P.off_loc[ns];
    t.n_dof = P.n_dof;
    c->n_alpha = ns * nrbm;

    // ---- device buffers ----
    c->L = c->alloc<double>(oL);
    c->Li = c->alloc<double>(std::max(1LL, oLi));
    c->Z = c->alloc<double>(oZ);
    c->S = c->alloc<double>(oS);
    c->F64 = c->alloc<double>(oF);
    c->sw64 = c->alloc<double>(oF);
    c->sw32 = c->alloc<float>(oF);
    c->swhi = c->alloc<__hip_bfloat16>(oF);
    c->swlo = c->alloc<__hip_bfloat16>(oF);
    c->Pk = c->alloc<double>(std::max(1LL, oPk));
    c->n_Pk = oPk;
    if (c->opts.precond_fp32) c->Pk32 = c->alloc<float>(std::max(1LL, oPk));
    c->ypart = c->alloc<double>(std::max<long long>(1, (long long)kPsMaxSplit * t.nb_tot));
    c->W1 = c->alloc<double>(oP);
    c->W2 = c->alloc<double>(oP);
    c->Kc = c->alloc<double>(oKc);
    c->Rb = c->alloc<double>(oR);
    c->Cit = c->alloc<double>(36ll * ns);
    c->tau = c->alloc<double>(ns);
    c->diag = c->alloc<double>(t.nloc_tot);
    c->rho = c->alloc<double>(P.n_el);
    c->Emod = c->alloc<double>(std::max<long long>(1, P.n_el));
    c->info = c->alloc<int>(ns + 8);
    if (t.max_line > 128) c->bt_ws = c->alloc<char>(bt_plane_ws_bytes(t));
    if (t.max_line > kSweepMaxLine && t.max_line <= kSweepBigLine) c->bt_T = c->alloc<double>(bt_plane_fwd_doubles(t));
    const int ncg = P.n_cg;
    // Kbar_cc: one dense block per design, 16-row tiles for the coarse solve
    long long kcc_sz = 0;
    c->hcblk.clear();
    std::vector<int> cg_blk(std::max(1, ncg), 0);
    std::vector<CoarseTile> ctiles;
    for (const DesignMeta& D : c->designs) {
        if (D.n_cg == 0) continue;
        const int b = (int)c->hcblk.size();
        c->hcblk.push_back(CoarseBlk{D.cg0, D.n_cg, kcc_sz});
        kcc_sz += (long long)D.n_cg * D.n_cg;
        for (int q = 0; q < D.n_cg; ++q) cg_blk[D.cg0 + q] = b;
        for (int r0 = 0; r0 < D.n_cg; r0 += 16) ctiles.push_back(CoarseTile{b, r0});
    }
    c->Kcc = c->alloc<double>(std::max(1LL, kcc_sz));
    c->Kcc_w = c->alloc<double>(std::max(1LL, kcc_sz));
    c->Kcc_inv = c->alloc<double>(std::max(1LL, kcc_sz));
    if (!c->hcblk.empty()) {
        std::vector<GemmDesc> gd;
        std::vector<PotrfDesc> pd;
        std::vector<TrsmDesc> td;
        for (const CoarseBlk& B : c->hcblk) {
            gd.push_back(GemmDesc{B.off, B.off, B.off, B.n, B.n, B.n, B.n, B.n, B.n});
            pd.push_back(PotrfDesc{B.off, B.n, B.n});
            td.push_back(TrsmDesc{B.off, B.off, B.n, B.n, B.n, B.n});
        }
        c->d_cc_gemm = c->upload(gd);
        c->d_cc_potrf = c->upload(pd);
        c->d_cc_trsm = c->upload(td);
        t.cblk = c->upload(c->hcblk);
        t.ctiles = c->upload(ctiles);
        t.n_ctiles = (int)ctiles.size();
    }
    t.cg_blk = c->upload(cg_blk);
    {
        std::vector<int> seg;
        for (const DesignMeta& D : c->designs) {
            seg.push_back(D.lam0);
            seg.push_back(D.n_lambda);
        }
        t.seg = c->upload(seg);
    }
    t.hkseg.clear();
    if (c->segmented) {
        std::vector<int> rb((size_t)std::max(1, P.n_lambda / 256), 0);
        for (int d = 0; d < (int)c->designs.size(); ++d) {
            const DesignMeta& D = c->designs[d];
            const int base = std::max(1, (int)std::llround(256.0 * D.n_rows / std::max(1, P.n_lambda)));
            t.hkseg.push_back(KrySeg{D.lam0, D.n_rows, base});
            for (int q = D.lam0 / 256; q < (D.lam0 + D.n_rows) / 256; ++q) rb[q] = d;
        }
        t.kseg = c->upload(t.hkseg);
        t.rb_design = c->upload(rb);
    }
    const int na = c->n_alpha;
    c->GG = c->alloc<double>((long long)na * na);
    c->GG_w = c->alloc<double>((long long)na * na);
    c->GG_inv = c->alloc<double>((long long)na * na);
    c->w = c->alloc<double>(2ll * P.n_lambda);
    c->bg_w = c->alloc<double>((long long)P.bg_row.size());

    // descriptors
    std::vector<GemmDesc> dsy(ns), dF(ns);
    std::vector<PotrfDesc> dpo(ns);
    std::vector<TrsmDesc> dtr(ns);
    for (int s = 0; s < ns; ++s) {
        const SubMeta& M = c->hsubs[s];
        dsy[s] = GemmDesc{M.off_Z, M.off_Z, M.off_S, M.n_beta, M.n_beta, M.n_i, M.n_beta, M.n_beta, M.n_beta};
        dF[s] = GemmDesc{M.off_P, M.off_P, M.off_F, M.n_b, M.n_b, M.n_b, M.n_b, M.n_b, M.ldF};
        dpo[s] = PotrfDesc{M.off_P, M.n_b, M.n_b};
        dtr[s] = TrsmDesc{M.off_P, M.off_P, M.n_b, M.n_b, M.n_b, M.n_b};
        const int tb = (M.n_beta + 63) / 64, tf = (M.n_b + 63) / 64;
        c->syrk_tdim = std::max(c->syrk_tdim, tb);
        c->F_tdim = std::max(c->F_tdim, tf);
        c->max_nb_cols = std::max(c->max_nb_cols, M.n_b);
    }
    c->d_syrk = c->upload(dsy);
    c->d_F = c->upload(dF);
    c->d_potrf = c->upload(dpo);
    c->d_trsm = c->upload(dtr);
    if (c->opts.defl_modes > 0 && P.n_lambda > 0) {
        const long long oPt = oP;
        std::vector<GemmDesc> dd(ns);
        for (int s = 0; s < ns; ++s) {
            const SubMeta& M = c->hsubs[s];
            dd[s] = GemmDesc{M.off_P, M.off_P, M.off_P, M.n_b, M.n_b, M.n_b, M.n_b, M.n_b, M.n_b};
        }
        c->d_df = c->upload(dd);
        c->dfL = c->alloc<double>(oPt);
        c->dfM = c->alloc<double>(oPt);
        c->dfB = c->alloc<double>(oPt);
        c->dfC = c->alloc<double>(oPt);
        c->dfOmega = c->alloc<double>(t.nb_tot);
        c->dfU = c->alloc<double>(8 * t.nb_tot);
        c->dfMu = c->alloc<double>((long long)ns * c->opts.defl_modes);
        c->dfCnt = c->alloc<int>(ns);
        c->dfCol0 = c->alloc<int>(ns);
        c->df_cap = (ns * c->opts.defl_modes + 63) / 64;
        const long long blk = (long long)P.n_lambda * 64;
        c->dfY = c->alloc<double>(blk * c->df_cap);
        double* wq = c->alloc<double>(2 * blk * c->df_cap);
        for (int b = 0; b < c->df_cap; ++b) {
            c->dfW.push_back(wq + blk * (2ll * b));
            c->dfQ.push_back(wq + blk * (2ll * b + 1));
        }
        c->dfW_dev = c->upload(std::vector<const double*>(c->dfW.begin(), c->dfW.end()));
        c->dfQ_dev = c->upload(std::vector<const double*>(c->dfQ.begin(), c->dfQ.end()));
        c->dfPsi = c->alloc<double>(4096ll * c->df_cap);
        c->dfPad = c->alloc<double>(blk);
    }
    c->rep_of.resize(ns);
    for (int s = 0; s < ns; ++s) c->rep_of[s] = s;
    c->n_setup_subs = ns;
    if (c->opts.recycle && c->designs.size() == 1) {
        c->h_dsy = dsy;
        c->h_dF = dF;
        c->h_dpo = dpo;
        c->h_dtr = dtr;
        c->d_syrk_r = c->alloc<GemmDesc>(ns);
        c->d_F_r = c->alloc<GemmDesc>(ns);
        c->d_potrf_r = c->alloc<PotrfDesc>(ns);
        c->d_trsm_r = c->alloc<TrsmDesc>(ns);
        c->subs_rep = c->alloc<SubMeta>(ns);
        c->hash_dev = c->alloc<unsigned long long>(ns);
        c->pair_dev = c->alloc<int>(2LL * ns);
        c->flag_dev = c->alloc<int>(ns);
        c->map_dev = c->alloc<int>(ns);
        c->rbm_tmp = c->alloc<double>(37LL * ns);
        // structural key: local grid, class sizes and the class and class index of every local
        // DOF (which fixes the interface order, the line blocks and the corner set)
        c->skey.assign(ns, 0);
        for (int s = 0; s < ns; ++s) {
            unsigned long long h = 1469598103934665603ull;
            auto put = [&](long long v) {
                h ^= (unsigned long long)v;
                h *= 1099511628211ull;
            };
            for (int a = 0; a < 3; ++a) put(P.nn[3 * s + a]);
            put(P.n_loc[s]);
            put(P.n_i[s]);
            put(P.n_b[s]);
            put(P.n_c[s]);
            put(P.band[s]);
            for (long long q = P.off_loc[s]; q < P.off_loc[s + 1]; ++q) {
                put(P.lcls[q]);
                put(P.lidx[q]);
            }
            c->skey[s] = h;
        }
    }
    const int nsmall = std::max(ncg, na);
    c->d_one = c->upload(std::vector<GemmDesc>{GemmDesc{0, 0, 0, nsmall, nsmall, nsmall, nsmall, nsmall, nsmall}});
    c->d_potrf_one = c->upload(std::vector<PotrfDesc>{PotrfDesc{0, nsmall, nsmall}});
    c->d_trsm_one = c->upload(std::vector<TrsmDesc>{TrsmDesc{0, 0, nsmall, nsmall, nsmall, nsmall}});


    // topology arrays
    std::vector<int> bq_s(t.nb_tot);
    for (int s = 0; s < ns; ++s)
        for (long long q = P.off_b[s]; q < P.off_b[s + 1]; ++q) bq_s[q] = s;
    c->subs_dev = c->upload(c->hsubs);
    t.subs = c->subs_dev;
    c->hsubs_act = c->hsubs;
    t.lines = c->upload(c->hlines);
    t.lcls = c->upload(P.lcls);
    t.lidx = c->upload(P.lidx);
    t.lglob = c->upload(P.lglob);
    t.lown = c->upload(P.lown);
    t.i_loc = c->upload(P.i_loc);
    t.b_loc = c->upload(P.b_loc);
    t.c_loc = c->upload(P.c_loc);
    t.c_glob = c->upload(P.c_glob);
    t.bq_s = c->upload(bq_s);
    t.row_s = c->upload(P.row_s);
    t.row_j = c->upload(P.row_j);
    t.row_sg = c->upload(P.row_sg);
    // absolute Y row of each (row, side): the scatter's loads need no subdomain lookup
    std::vector<long long> yo(P.row_s.size());
    for (size_t e = 0; e < yo.size(); ++e) yo[e] = P.row_s[e] >= 0 ? c->hsubs[P.row_s[e]].off_b + P.row_j[e] : -1;
    t.row_yo = c->upload(yo);
    if (P.method == FETI_DP && P.n_cg > 0 && P.n_lambda > 0) {
        // coarse fold entries of every lambda row (values follow at each setup: launch_fold_rows)
        int W = 0;
        for (int r = 0; r < P.n_lambda; ++r) {
            int ne = 0;
            for (int e = 0; e < 2; ++e)
                if (P.row_s[2 * r + e] >= 0) ne += c->hsubs[P.row_s[2 * r + e]].n_c;
            W = std::max(W, ne);
        }
        W = std::max(W, 1);
        std::vector<int> fn(P.n_lambda, 0), fc((size_t)P.n_lambda * W, 0);
        for (int r = 0; r < P.n_lambda; ++r) {
            int ne = 0;
            for (int e = 0; e < 2; ++e) {
                const int s = P.row_s[2 * r + e];
                if (s < 0) continue;
                const SubMeta& M = c->hsubs[s];
                for (int q = 0; q < M.n_c; ++q) fc[(size_t)r * W + ne++] = P.c_glob[M.off_c + q];
            }
            fn[r] = ne;
        }
        t.fr_w = W;
        t.fr_n = c->upload(fn);
        t.fr_col = c->upload(fc);
        t.fr_val = c->alloc<double>((long long)P.n_lambda * W);
        // rows grouped by their pair of subdomains: each group's corner DOFs (the union over both
        // sides) are staged once, and fr_pos places every fold entry in that union
        std::map<std::pair<int, int>, std::vector<int>> groups;
        for (int r = 0; r < P.n_lambda; ++r) groups[{P.row_s[2 * r], P.row_s[2 * r + 1]}].push_back(r);
        std::vector<int> pr_ptr{0}, pu_ptr{0}, pu_cg, fpos((size_t)P.n_lambda * W, 0), ipos(P.n_lambda);
        std::vector<int4> prec;
        int maxu = 0;
        for (auto& g : groups) {
            std::vector<int> U;
            for (int r : g.second)
                for (int e = 0; e < fn[r]; ++e) U.push_back(fc[(size_t)r * W + e]);
            std::sort(U.begin(), U.end());
            U.erase(std::unique(U.begin(), U.end()), U.end());
            maxu = std::max(maxu, (int)U.size());
            for (int r : g.second) {
                const size_t i = prec.size();
                ipos[r] = (int)i;
                const int fl = fn[r] << 2 | (P.row_sg[2 * (size_t)r] < 0) | (P.row_sg[2 * (size_t)r + 1] < 0) << 1;
                prec.push_back(int4{(int)yo[2 * (size_t)r], (int)yo[2 * (size_t)r + 1], fl, r});
                for (int e = 0; e < fn[r]; ++e)
                    fpos[i * W + e] = (int)(std::lower_bound(U.begin(), U.end(), fc[(size_t)r * W + e]) - U.begin());
            }
            pr_ptr.push_back((int)prec.size());
            pu_cg.insert(pu_cg.end(), U.begin(), U.end());
            pu_ptr.push_back((int)pu_cg.size());
        }
        // local product rows are stored as int in the row records. The pair form sums a row's fold
        // entries one at a time and runs a group's rows in one workgroup, so it pays only for
        // narrow rows in long groups: 2D with 126-row groups (27.5 us at 16x16 subdomains of 64^2
        // against 58 us for the fold per subdomain, then the scatter; solve 54.4 against 56.0 ms).
        // 3D rows carry up to 48 entries (145 us at 4x4x4 subdomains against 84 us), and the
        // batched 2D designs have groups of 30-94 rows (solve 152.4 against 148.2 ms): both take
        // the two kernels.
        const bool long_groups = (long long)P.n_lambda >= (long long)kFoldPairMinRows * (long long)groups.size();
        if (maxu <= kFoldPairMaxU && W <= kFoldPairMaxW && long_groups && t.nb_tot < (1LL << 31)) {
            t.n_pairs = (int)groups.size();
            t.pr_ptr = c->upload(pr_ptr);
            t.pu_ptr = c->upload(pu_ptr);
            for (int e = 0; e < 4; ++e) pu_cg.push_back(0);   // 4-entry index loads near the end
            t.pu_cg = c->upload(pu_cg);
            t.fr_pos = c->upload(fpos);
            for (int e = 0; e < kFoldRows; ++e) prec.push_back(int4{-1, -1, 0, 0});   // a pass's last records
            t.pr_rec = c->upload(prec);
            t.pr_ipos = c->upload(ipos);
            t.pr_fval = c->alloc<double>((long long)P.n_lambda * W);
        }
    }
    t.row_sh = c->upload(P.row_sh);
    t.sh_ptr = c->upload(P.sh_ptr);
    t.sh_s = c->upload(P.sh_s);
    t.sh_l = c->upload(P.sh_l);
    {
        int R = 1;
        for (long long q = 0; q < t.nb_tot; ++q) R = std::max(R, P.bg_ptr[q + 1] - P.bg_ptr[q]);
        std::vector<int> gm((size_t)std::max<long long>(1, t.nb_tot) * R, 0);
        for (long long q = 0; q < t.nb_tot; ++q)
            for (int e = P.bg_ptr[q], u = 0; e < P.bg_ptr[q + 1]; ++e, ++u)
                gm[q * R + u] = P.bg_sg[e] > 0 ? P.bg_row[e] + 1 : -(P.bg_row[e] + 1);
        t.gmap = c->upload(gm);
        t.gmap_R = R;
    }
    if (t.max_nc > 32) throw std::runtime_error("more than 32 corner DOFs in one subdomain");
    {   // preconditioner workgroups: at most one per CU in all; parts go one at a time to the
        // subdomain with the most packed tiles per workgroup (at most kPsMaxSplit parts each)
        std::vector<int> G(ns, 1), nt(ns);
        for (int s = 0; s < ns; ++s) {
            const int nT = (c->hsubs[s].n_b + 63) / 64;
            nt[s] = nT * (nT + 1) / 2;
        }
        int total = ns;
        while (total < 256) {
            int best = -1;
            for (int s = 0; s < ns; ++s)
                if (G[s] < kPsMaxSplit && nt[s] > G[s] &&
                    (best < 0 || (long long)nt[s] * G[best] > (long long)nt[best] * G[s]))
                    best = s;
            if (best < 0) break;
            ++G[best];
            ++total;
        }
        std::vector<int4> wk;
        t.ps_maxG = 1;
        for (int s = 0; s < ns; ++s) {
            t.ps_maxG = std::max(t.ps_maxG, G[s]);
            for (int g = 0; g < G[s]; ++g) wk.push_back(int4{s, g, G[s], 0});
        }
        // longest parts first
        std::stable_sort(wk.begin(), wk.end(), [&](const int4& a, const int4& b) {
            return (long long)nt[a.x] * b.z > (long long)nt[b.x] * a.z;
        });
        t.ps_work = c->upload(wk);
        t.ps_G = c->upload(G);
        t.ps_nwg = (int)wk.size();
    }
    t.bg_ptr = c->upload(P.bg_ptr);
    t.bg_row = c->upload(P.bg_row);
    t.bg_sg = c->upload(P.bg_sg);
    t.cc_ptr = c->upload(P.cc_ptr);
    t.cc_s = c->upload(P.cc_s);
    t.cc_j = c->upload(P.cc_j);
    for (int a = 0; a < 3; ++a) {
        t.ax_first[a] = c->upload(P.ax_first[a]);
        t.ax_cnt[a] = c->upload(P.ax_cnt[a]);
    }
    t.dsg.clear();
    for (const DesignMeta& D : c->designs) {
        DesignDev E;
        E.sub0 = D.sub0;
        E.lam0 = D.lam0;
        E.n_lambda = D.n_lambda;
        E.el0 = D.el0;
        E.n_el = D.n_el;
        E.dof0 = D.dof0;
        E.n_dof = D.n_dof;
        for (int a = 0; a < 3; ++a) {
            E.nel[a] = D.nel[a];
            E.nsub[a] = D.nsub[a];
            E.axf[a] = c->upload(D.ax_first[a]);
            E.axc[a] = c->upload(D.ax_cnt[a]);
        }
        t.dsg.push_back(E);
    }
    build_fl_tiles(c);
    c->pivdev = c->alloc<double>(ns);
    std::vector<double> K0 = element_K0(P.dim, P.nu);
    c->K0dev = c->upload(K0);
    t.K0dev = c->K0dev;
    CHECK_LAUNCH();

    // solve buffers
    const long long nl = std::max(1, P.n_lambda);
    const long long nbk = std::max<long long>(1, t.nb_tot), nck = std::max<long long>(1, t.nc_tot);
    c->f_last = c->alloc<double>(P.n_dof);
    c->fi = c->alloc<double>(t.ni_tot);
    c->fbeta = c->alloc<double>(t.nb_tot + t.nc_tot);
    c->h = c->alloc<double>(t.ni_tot);
    c->g = c->alloc<double>(t.nb_tot + t.nc_tot);
    c->yb = c->alloc<double>(nbk);
    c->yc = c->alloc<double>(nck);
    c->fbar_s = c->alloc<double>(nck);
    c->Tsum = c->alloc<double>(nck);
    c->d = c->alloc<double>(nl);
    c->lam0 = c->alloc<double>(nl);
    c->lam = c->alloc<double>(nl);
    c->lt = c->alloc<double>(nl);
    c->lt2 = c->alloc<double>(nl);
    c->lam_prev = c->alloc<double>(nl);
    c->r = c->alloc<double>(nl);
    c->zv = c->alloc<double>(nl);
    c->tmpv = c->alloc<double>(nl);
    c->xb = c->alloc<double>(nbk);
    c->ubeta = c->alloc<double>(t.nb_tot + t.nc_tot);
    c->ui = c->alloc<double>(t.ni_tot);
    c->uloc = c->alloc<double>(t.nloc_tot);
    c->uc = c->alloc<double>(std::max(1, ncg));
    c->alpha = c->alloc<double>(std::max(1, na));
    c->e = c->alloc<double>(std::max(1, na));
    c->GY = c->alloc<double>((long long)std::max(1, na) * kMaxDirs);
    c->tcoef = c->alloc<double>((long long)std::max(1, na) * kMaxDirs);
    c->u_int = c->alloc<double>(P.n_dof);
    c->Ybuf = c->alloc<double>(nbk * kMaxDirs);
    c->Tbuf = c->alloc<double>(nck * kMaxDirs);
    c->vbuf = c->alloc<double>((long long)std::max(1, ncg) * kMaxDirs);
    c->Qtmp = c->alloc<double>(nl * kMaxDirs);
    c->Zk = c->alloc<double>(nl * kMaxDirs);
    c->Qk = c->alloc<double>(nl * kMaxDirs);
    const int nsegd = c->segmented ? (int)c->designs.size() : 1;   // per-design k x k blocks
    c->Delta = c->alloc<double>((long long)nsegd * kMaxDirs * kMaxDirs);
    c->Tm = c->alloc<double>((long long)nsegd * kMaxDirs * kMaxDirs);
    c->gam = c->alloc<double>((long long)nsegd * kMaxDirs);
    c->part = c->alloc<double>(kGramPartCap);
    const int nd = (int)c->designs.size();
    // [16 + d]: per-design dots; segmented: [16 + nd + d] kept-column masks, [16 + 2 nd + d] ranks
    c->scal = c->alloc<double>(16 + 3 * nd);
    c->rank_dev = reinterpret_cast<int*>(c->scal + 8);
    HIPCHK(hipHostMalloc((void**)&c->hpin, sizeof(double) * (16 + 3 * nd), hipHostMallocDefault));
    for (int q = 0; q < 2; ++q) {
        HIPCHK(hipHostMalloc((void**)&c->hslot[q], sizeof(double) * (16 + 3 * nd + 2),
                             hipHostMallocMapped | hipHostMallocCoherent));
        std::memset(c->hslot[q], 0, sizeof(double) * (16 + 3 * nd + 2));
        HIPCHK(hipHostGetDevicePointer((void**)&c->hslot_dev[q], c->hslot[q], 0));
    }
    c->eps0_d.assign(nd, 0.0);
    c->true_d.assign(nd, 0.0);
    c->qk_ptr = c->upload(std::vector<const double*>{c->Qk});
    c->zk_ptr = c->upload(std::vector<const double*>{c->Zk});
    c->tcbuf = c->alloc<double>((long long)std::max(1, ncg) * kMaxDirs);
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
}

void check_info(feti_ctx* c, int n, const char* what);

// Round-off test of the reduced-precision operator, per subdomain: factorise F_s and its
// rounding to the context's precision in FP64; a subdomain keeps the reduced precision only
// if every Cholesky pivot agrees to 2 percent (otherwise rounding has reached the smallest
// eigenvalues of F_s and its tiles run in FP64).
// ts / dpo: the subdomains set up (all, or the representatives of the module types); ci[s]:
// the position in ts of subdomain s's representative.
void classify_precision(feti_ctx* c, const DevTopo& ts, const PotrfDesc* dpo, const std::vector<int>& ci) {
    const DevTopo& t = c->t;
    hipStream_t st = c->st;
    c->hybrid = false;
    c->n_fp64_subs = 0;
    if (c->opts.precision == FETI_FP64 || c->P.method != FETI_DP) return;
    const int nr = ts.n_sub;
    launch_copy_F_rounded(ts, c->F64, FETI_FP64, c->W1, st);
    launch_copy_F_rounded(ts, c->F64, c->opts.precision, c->W2, st);
    HIPCHK(hipMemsetAsync(c->info, 0, sizeof(int) * (t.n_sub + 8), st));
    launch_potrf(dpo, nr, t.max_nb, c->W1, c->info, st);
    CHECK_LAUNCH();
    check_info(c, nr, "Cholesky of F_s");
    HIPCHK(hipMemsetAsync(c->info, 0, sizeof(int) * (t.n_sub + 8), st));
    launch_potrf(dpo, nr, t.max_nb, c->W2, c->info, st);
    launch_pivot_compare(ts, c->W1, c->W2, c->info, c->pivdev, st);
    CHECK_LAUNCH();
    std::vector<double> dev(nr);
    HIPCHK(hipMemcpyAsync(dev.data(), c->pivdev, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int>& ok = c->sub_ok;
    ok.assign(t.n_sub, 0);
    for (int s = 0; s < t.n_sub; ++s) {
        ok[s] = dev[ci[s]] <= 2e-2 ? 1 : 0;
        c->n_fp64_subs += 1 - ok[s];
    }
    if (verbose()) {
        std::vector<double> d2 = dev;
        std::sort(d2.begin(), d2.end());
        fprintf(stderr, "[feti] round-off metric quantiles: 50%% %.2e 80%% %.2e 90%% %.2e 95%% %.2e max %.2e\n",
                d2[d2.size() / 2], d2[d2.size() * 8 / 10], d2[d2.size() * 9 / 10], d2[d2.size() * 95 / 100], d2.back());
    }
    c->hybrid = true;
    build_fl_tiles(c);
}

struct Timer {
    feti_ctx* c;
    int slot;
    Timer(feti_ctx* c_, int s) : c(c_), slot(s) { HIPCHK(hipEventRecord(c->ev[0], c->st)); }
    void stop() {
        HIPCHK(hipEventRecord(c->ev[1], c->st));
        HIPCHK(hipEventSynchronize(c->ev[1]));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        c->last_ms[slot] = ms;
    }
};

void check_info(feti_ctx* c, int n, const char* what) {
    std::vector<int> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), c->info, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int i = 0; i < n; ++i)
        if (h[i]) {
            char buf[160];
            snprintf(buf, sizeof buf, "%s: non-positive pivot (matrix %d, row %d)", what, i, h[i] - 1);
            throw std::runtime_error(buf);
        }
}

// Dense SPD n x n matrix A (device) -> Ainv (device), via Cholesky, X = L^{-1}, Ainv = X^T X.
void dense_spd_inverse(feti_ctx* c, int n, const double* A, double* work, double* Ainv, const char* what) {
    if (n == 0) return;
    std::vector<GemmDesc> gd{GemmDesc{0, 0, 0, n, n, n, n, n, n}};
    std::vector<PotrfDesc> pd{PotrfDesc{0, n, n}};
    std::vector<TrsmDesc> td{TrsmDesc{0, 0, n, n, n, n}};
    HIPCHK(hipMemcpyAsync(c->d_one, gd.data(), sizeof(GemmDesc), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->d_potrf_one, pd.data(), sizeof(PotrfDesc), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->d_trsm_one, td.data(), sizeof(TrsmDesc), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(work, A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemsetAsync(c->info, 0, sizeof(int), c->st));
    launch_potrf(c->d_potrf_one, 1, n, work, c->info, c->st);
    CHECK_LAUNCH();
    check_info(c, 1, what);
    launch_set_identity(Ainv, n, n, c->st);
    launch_trsm_identity(c->d_trsm_one, 1, n, work, Ainv, c->st);
    // Ainv currently holds X = L^{-1}; form X^T X into work, then copy
    launch_gemm_tn(c->d_one, 1, (n + 63) / 64, Ainv, Ainv, work, 1.0, 0.0, 1, c->st);
    CHECK_LAUNCH();
    HIPCHK(hipMemcpyAsync(Ainv, work, sizeof(double) * n * n, hipMemcpyDeviceToDevice, c->st));
}

// Kbar_cc^{-1}, block by block (one dense block per design): Cholesky, L^{-1} by a triangular
// solve on the identity, then L^{-T} L^{-1}, each step one batched launch over the blocks.
void coarse_inverse(feti_ctx* c) {
    const std::vector<CoarseBlk>& B = c->hcblk;
    const int nb = (int)B.size();
    if (nb == 0) return;
    const long long sz = B.back().off + (long long)B.back().n * B.back().n;
    int maxn = 0;
    for (const CoarseBlk& b : B) maxn = std::max(maxn, b.n);
    hipStream_t st = c->st;
    HIPCHK(hipMemcpyAsync(c->Kcc_w, c->Kcc, sizeof(double) * sz, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(c->info, 0, sizeof(int) * nb, st));
    launch_potrf(c->d_cc_potrf, nb, maxn, c->Kcc_w, c->info, st);
    CHECK_LAUNCH();
    check_info(c, nb, "coarse Cholesky");
    for (const CoarseBlk& b : B) launch_set_identity(c->Kcc_inv + b.off, b.n, b.n, st);
    launch_trsm_identity(c->d_cc_trsm, nb, maxn, c->Kcc_w, c->Kcc_inv, st);
    launch_gemm_tn(c->d_cc_gemm, nb, (maxn + 63) / 64, c->Kcc_inv, c->Kcc_inv, c->Kcc_w, 1.0,
                   0.0, 1, st);
    CHECK_LAUNCH();
    HIPCHK(hipMemcpyAsync(c->Kcc_inv, c->Kcc_w, sizeof(double) * sz, hipMemcpyDeviceToDevice, st));
}

// Module types (opts.recycle, single design): subdomains with the same structural key and the
// same densities share their factorisation and local operators, as the paper's modular designs
// recycle one factorisation per module type (Sec. 1; Sec. 2.1). Densities are compared through a
// device hash per subdomain, and every candidate pair element by element. Returns the
// representatives (ascending); rep_of[s] names each subdomain's.
std::vector<int> find_modules(feti_ctx* c) {
    const int ns = c->P.n_sub;
    std::vector<int>& rep = c->rep_of;
    rep.resize(ns);
    for (int s = 0; s < ns; ++s) rep[s] = s;
    if (c->opts.recycle && c->designs.size() == 1 && ns > 1) {
        hipStream_t st = c->st;
        launch_rho_hash(c->t, c->rho, c->hash_dev, st);
        CHECK_LAUNCH();
        std::vector<unsigned long long> h(ns);
        HIPCHK(hipMemcpyAsync(h.data(), c->hash_dev, sizeof(unsigned long long) * ns, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::map<std::pair<unsigned long long, unsigned long long>, int> first;
        std::vector<int> pairs;
        for (int s = 0; s < ns; ++s) {
            auto it = first.emplace(std::make_pair(c->skey[s], h[s]), s).first;
            if (it->second != s) {
                pairs.push_back(s);
                pairs.push_back(it->second);
            }
        }
        const int np = (int)pairs.size() / 2;
        if (np > 0) {
            HIPCHK(hipMemcpyAsync(c->pair_dev, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice, st));
            launch_rho_match(c->t, c->rho, c->pair_dev, np, c->flag_dev, st);
            CHECK_LAUNCH();
            std::vector<int> flag(np);
            HIPCHK(hipMemcpyAsync(flag.data(), c->flag_dev, sizeof(int) * np, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int q = 0; q < np; ++q)
                if (!flag[q]) rep[pairs[2 * q]] = pairs[2 * q + 1];
        }
    }
    std::vector<int> reps;
    for (int s = 0; s < ns; ++s)
        if (rep[s] == s) reps.push_back(s);
    c->n_setup_subs = (int)reps.size();
    return reps;
}

// Assembly, factorisation and explicit local operators for the current densities.
void build_deflation(feti_ctx* c);

void numeric_setup(feti_ctx* c) {
    c->drop_graphs();
    Timer tm(c, 2);
    const Plan& P = c->P;
    DevTopo& t = c->t;
    hipStream_t st = c->st;
    const auto& H = c->hsubs;
    const int ns = P.n_sub;
    auto zero = [&](void* p, long long bytes) {
        if (bytes > 0) HIPCHK(hipMemsetAsync(p, 0, bytes, st));
    };
    long long nL = 0, nZ = 0, nS = 0, nF = 0;
    if (!H.empty()) {
        const SubMeta& Ml = H.back();
        const LineMeta& Ll = c->hlines.back();
        nL = Ll.off_sub + (long long)Ll.n * Ll.n_prev;
        nZ = Ml.off_Z + (long long)Ml.n_i * Ml.n_beta;
        nS = Ml.off_S + (long long)Ml.n_beta * Ml.n_beta;
        nF = Ml.off_F + (long long)Ml.rows_F * Ml.ldF;
    }
    // every subdomain back on its own storage before the assembly
    if (c->aliased) {
        HIPCHK(hipMemcpyAsync(c->subs_dev, H.data(), sizeof(SubMeta) * ns, hipMemcpyHostToDevice, st));
        c->hsubs_act = H;
        c->aliased = false;
    }
    zero(c->L, nL * 8);
    zero(c->Z, nZ * 8);
    zero(c->S, nS * 8);
    zero(c->F64, nF * 8);
    zero(c->diag, t.nloc_tot * 8);
    zero(c->info, (t.n_sub + 8) * 4);
    // every subdomain is assembled (its diagonal feeds the scaling weights); the factorisation
    // and the local operators are formed for the representatives only (ts, nr)
    launch_simp_moduli(P.n_el, c->rho, c->p, c->E0, c->Emin, c->Emod, st);
    launch_assemble(t, c->Emod, c->L, c->Z, c->S, c->diag, st);
    CHECK_LAUNCH();
    const std::vector<int> reps = find_modules(c);
    const int nr = (int)reps.size();
    DevTopo ts = t;
    const GemmDesc *dsy = c->d_syrk, *dF = c->d_F;
    const PotrfDesc* dpo = c->d_potrf;
    const TrsmDesc* dtr = c->d_trsm;
    if (nr < ns) {
        std::vector<SubMeta> hr(nr);
        std::vector<GemmDesc> a(nr), b(nr);
        std::vector<PotrfDesc> pp(nr);
        std::vector<TrsmDesc> tt(nr);
        for (int i = 0; i < nr; ++i) {
            hr[i] = H[reps[i]];
            a[i] = c->h_dsy[reps[i]];
            b[i] = c->h_dF[reps[i]];
            pp[i] = c->h_dpo[reps[i]];
            tt[i] = c->h_dtr[reps[i]];
        }
        HIPCHK(hipMemcpyAsync(c->subs_rep, hr.data(), sizeof(SubMeta) * nr, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->d_syrk_r, a.data(), sizeof(GemmDesc) * nr, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->d_F_r, b.data(), sizeof(GemmDesc) * nr, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->d_potrf_r, pp.data(), sizeof(PotrfDesc) * nr, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->d_trsm_r, tt.data(), sizeof(TrsmDesc) * nr, hipMemcpyHostToDevice, st));
        ts.subs = c->subs_rep;
        ts.n_sub = nr;
        dsy = c->d_syrk_r;
        dF = c->d_F_r;
        dpo = c->d_potrf_r;
        dtr = c->d_trsm_r;
    }
    launch_bt_factor_li(ts, c->L, c->Li, c->info, c->bt_ws, st);
    CHECK_LAUNCH();
    check_info(c, nr, "interior Cholesky");
    launch_bt_invert(t, c->L, c->Li, st);
    CHECK_LAUNCH();
    if (c->bt_T)
        launch_bt_forward_planes(ts, c->L, c->Li, c->Z, c->bt_T, st);
    else
        launch_bt_forward_li(ts, c->L, c->Li, c->Z, st);
    CHECK_LAUNCH();
    if (c->opts.precond == FETI_LUMPED || c->opts.precond == FETI_SUPERLUMPED) launch_pack_sym(ts, c->S, c->Pk, st);
    if (c->opts.precond == FETI_SUPERLUMPED) launch_pk_diag_only(ts, c->Pk, st);
    launch_gemm_tn(dsy, nr, c->syrk_tdim, c->Z, c->Z, c->S, -1.0, 1.0, 1, st);
    CHECK_LAUNCH();
    if (c->opts.precond == FETI_DIRICHLET) launch_pack_sym(ts, c->S, c->Pk, st);
    if (c->Pk32) launch_round_f32(c->n_Pk, c->Pk, c->Pk32, st);
    if (P.method == FETI_TFETI)
        launch_tfeti_rbm(ts, c->S, c->Rb, c->Cit, c->tau, c->W1, st);
    else
        launch_copy_Sbb(ts, c->S, c->W1, 0, st);
    CHECK_LAUNCH();
    zero(c->info, (t.n_sub + 8) * 4);
    launch_potrf(dpo, nr, t.max_nb, c->W1, c->info, st);
    CHECK_LAUNCH();
    check_info(c, nr, "interface Schur complement Cholesky");
    launch_copy_Sbb(ts, c->S, c->W2, 1, st);
    launch_trsm_identity(dtr, nr, c->max_nb_cols, c->W1, c->W2, st);
    launch_gemm_tn(dF, nr, c->F_tdim, c->W2, c->W2, c->F64, 1.0, 0.0, 1, st);
    CHECK_LAUNCH();
    if (P.method == FETI_TFETI)
        launch_tfeti_fix(ts, c->Rb, c->tau, c->F64, st);
    else
        launch_frc(ts, c->S, c->F64, c->Kc, st);
    CHECK_LAUNCH();
    launch_swizzle(ts, c->F64, c->sw64, c->sw32, c->swhi, c->swlo, st);
    CHECK_LAUNCH();
    std::vector<int> ci(ns, 0);   // compacted index of each subdomain's representative
    {
        std::vector<int> pos(ns, -1);
        for (int i = 0; i < nr; ++i) pos[reps[i]] = i;
        for (int s = 0; s < ns; ++s) ci[s] = pos[c->rep_of[s]];
    }
    if (nr < ns) {
        // members take their representative's operator storage; the per-subdomain Total FETI
        // results written by compacted index are spread to every subdomain
        std::vector<SubMeta>& A = c->hsubs_act;
        A = H;
        for (int s = 0; s < ns; ++s) {
            const SubMeta& R = H[c->rep_of[s]];
            SubMeta& M = A[s];
            M.line0 = R.line0;
            M.off_L = R.off_L;
            M.off_Z = R.off_Z;
            M.off_S = R.off_S;
            M.off_F = R.off_F;
            M.off_Fsw = R.off_Fsw;
            M.off_P = R.off_P;
            M.off_Pk = R.off_Pk;
            M.off_Kc = R.off_Kc;
            M.off_R = R.off_R;
        }
        HIPCHK(hipMemcpyAsync(c->subs_dev, A.data(), sizeof(SubMeta) * ns, hipMemcpyHostToDevice, st));
        c->aliased = true;
        if (P.method == FETI_TFETI) {
            HIPCHK(hipMemcpyAsync(c->map_dev, ci.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(c->rbm_tmp, c->Cit, sizeof(double) * 36 * nr, hipMemcpyDeviceToDevice, st));
            launch_gather_rows(ns, 36, c->map_dev, c->rbm_tmp, c->Cit, st);
            HIPCHK(hipMemcpyAsync(c->rbm_tmp, c->tau, sizeof(double) * nr, hipMemcpyDeviceToDevice, st));
            launch_gather_rows(ns, 1, c->map_dev, c->rbm_tmp, c->tau, st);
            CHECK_LAUNCH();
        }
    }
    if (P.method == FETI_DP) launch_fold_rows(t, c->F64, st);
    launch_weights(t, c->opts.scaling == FETI_KSCALE, c->diag, c->w, c->bg_w, st);
    CHECK_LAUNCH();
    classify_precision(c, ts, dpo, ci);
    if (P.method == FETI_DP && P.n_cg > 0) {
        const CoarseBlk& last = c->hcblk.back();
        zero(c->Kcc, (last.off + (long long)last.n * last.n) * 8);
        launch_coarse_assemble(t, c->Kc, c->Kcc, st);
        CHECK_LAUNCH();
        coarse_inverse(c);
    }
    if (P.method == FETI_TFETI && c->n_alpha > 0) {
        zero(c->GG, (long long)c->n_alpha * c->n_alpha * 8);
        launch_ggt_assemble(t, c->Rb, c->GG, st);
        CHECK_LAUNCH();
        dense_spd_inverse(c, c->n_alpha, c->GG, c->GG_w, c->GG_inv, "G G^T Cholesky");
    }
    build_deflation(c);
    tm.stop();
}

// ---------------------------------------------------------------- operator applications

// Q = F Lambda (n_lambda x k) in the given precision. A reduced precision uses the
// per-subdomain selection of the setup (FP64 tiles for the subdomains that failed the
// round-off test, FP64 outputs) unless `pure` forces every tile to the reduced precision.
// Work buffers of one F*Lambda: local products Y (nb_tot x k), corner rows T (nc_tot x k), the
// coarse right-hand sides t and the coarse solution v (n_cg x k each).
struct FlBufs {
    void *Y, *T;
    double *v, *tc;
};

// Bytes of FlBufs for k columns laid out back to back, each part 256-byte aligned.
long long fl_bufs_bytes(const DevTopo& t, int k) {
    auto up = [](long long b) { return (b + 255) / 256 * 256; };
    const long long ncg = std::max(1, t.n_cg);
    return up(8LL * std::max<long long>(1, t.nb_tot) * k) + up(8LL * std::max<long long>(1, t.nc_tot) * k) +
           2 * up(8LL * ncg * k);
}

FlBufs fl_bufs_in(const DevTopo& t, int k, void* base) {
    auto up = [](long long b) { return (b + 255) / 256 * 256; };
    const long long ncg = std::max(1, t.n_cg);
    unsigned char* p = static_cast<unsigned char*>(base);
    FlBufs b;
    b.Y = p;
    p += up(8LL * std::max<long long>(1, t.nb_tot) * k);
    b.T = p;
    p += up(8LL * std::max<long long>(1, t.nc_tot) * k);
    b.tc = reinterpret_cast<double*>(p);
    p += up(8LL * ncg * k);
    b.v = reinterpret_cast<double*>(p);
    return b;
}

void apply_F_with(feti_ctx* c, int k, int prec, const double* Lam, double* Q, const FlBufs& b, bool time_it,
                  bool pure) {
    DevTopo& t = c->t;
    hipStream_t st = c->st;
    const void* A = prec == FETI_FP32 ? (const void*)c->sw32 : prec == FETI_BF16X3 ? (const void*)c->swhi : nullptr;
    const bool hyb = prec != FETI_FP64 && !pure && c->hybrid && prec == c->opts.precision;
    const int f32 = prec != FETI_FP64 && !hyb;
    if (time_it) HIPCHK(hipEventRecord(c->ev[2], st));
    if (hyb) {
        launch_flambda(t, prec, k, Lam, A, c->swlo, c->sw64, b.Y, b.T, st, &c->fl_hyb, 1);
    }
    else
        launch_flambda(t, prec, k, Lam, A, c->swlo, c->sw64, b.Y, b.T, st);
    CHECK_LAUNCH();
    if (time_it) HIPCHK(hipEventRecord(c->ev[3], st));
    if (c->P.method == FETI_DP && c->P.n_cg > 0) {
        launch_coarse(t, k, f32, b.T, nullptr, c->Kcc_inv, 1.0, b.v, b.tc, st);
        if (k >= 32 && t.n_pairs == 0) {   // wide fold rows (3D): the fold per subdomain, then the scatter
            launch_fold_coarse(t, k, f32, c->F64, b.v, b.Y, st);
            launch_scatter(t, k, f32, b.Y, Q, st);
        } else {
            launch_scatter_fold(t, k, f32, b.Y, b.v, Q, st);
        }
    } else {
        launch_scatter(t, k, f32, b.Y, Q, st);
    }
    CHECK_LAUNCH();
}

void apply_F(feti_ctx* c, int k, int prec, const double* Lam, double* Q, bool time_it = false, bool pure = false) {
    apply_F_with(c, k, prec, Lam, Q, FlBufs{c->Ybuf, c->Tbuf, c->vbuf, c->tcbuf}, time_it, pure);
}

// body() as a captured graph replayed on c->st (opts.graphs and a non-null stream), captured on
// first use for the given key; otherwise body() is launched directly.
template <class F>
void run_graph(feti_ctx* c, feti_ctx::GraphSlot& gs, int key, F&& body) {
    if (!c->opts.graphs || c->st == nullptr) {
        body();
        return;
    }
    if (!gs.e || gs.key != key) {
        if (gs.e) HIPCHK(hipGraphExecDestroy(gs.e));
        if (gs.g) HIPCHK(hipGraphDestroy(gs.g));
        gs = feti_ctx::GraphSlot{};
        HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
        body();
        HIPCHK(hipStreamEndCapture(c->st, &gs.g));
        HIPCHK(hipGraphInstantiate(&gs.e, gs.g, nullptr, nullptr, 0));
        gs.key = key;
    }
    HIPCHK(hipGraphLaunch(gs.e, c->st));
}

void project(feti_ctx* c, int k, double* Y) {
    if (c->P.method != FETI_TFETI || c->P.n_lambda == 0) return;
    DevTopo& t = c->t;
    launch_proj_G(t, k, Y, c->Rb, c->GY, c->st);
    launch_small_gemm(c->n_alpha, k, c->n_alpha, c->GG_inv, c->GY, c->tcoef, 1.0, c->st);
    launch_proj_apply(t, k, c->tcoef, c->Rb, 1.0, Y, c->st);
    CHECK_LAUNCH();
}

// use_f32: a pass on the reduced-precision operator, which applies the FP32 copy of the blocks
// when the context keeps one (opts.precond_fp32)
void precondition(feti_ctx* c, const double* r, double* Z, int one_column, int use_f32) {
    DevTopo& t = c->t;
    if (c->opts.precond == FETI_SUPERLUMPED)
        launch_precond_diag(t, r, c->bg_w, c->Pk, c->yb, c->st);
    else if (use_f32 && c->Pk32)
        launch_precond_local32(t, r, c->bg_w, c->Pk32, c->ypart, c->yb, c->st);
    else
        launch_precond_local(t, r, c->bg_w, c->Pk, c->ypart, c->yb, c->st);
    launch_precond_scatter(t, one_column, c->w, c->yb, Z, c->st);
    CHECK_LAUNCH();
}

// Wait for the stream by polling: the Krylov loop waits once per iteration for a few scalars,
// and a polling host resumes launching sooner than a blocking wait.
void wait_poll(feti_ctx* c) {
    hipError_t e;
    while ((e = hipStreamQuery(c->st)) == hipErrorNotReady) {
    }
    HIPCHK(e);
}

double read_scalar(feti_ctx* c, const double* dptr) {
    double v = 0;
    HIPCHK(hipMemcpyAsync(c->hpin, dptr, sizeof(double), hipMemcpyDeviceToHost, c->st));
    wait_poll(c);
    v = c->hpin[0];
    return v;
}

// scal[0 .. 16 + designs) to the host; returns scal[0]
double read_scalars(feti_ctx* c) {
    HIPCHK(hipMemcpyAsync(c->hpin, c->scal, sizeof(double) * (16 + c->designs.size()), hipMemcpyDeviceToHost, c->st));
    wait_poll(c);
    return c->hpin[0];
}

// Convergence with several designs is per design: each ratio sqrt(r_d^T z_d) / eps0_d (from
// the segmented dots in scal[16 + d], read by the last read_scalars) must reach tol; with one
// design it is the plain eps <= tol eps0.
bool converged(feti_ctx* c, double eps, double eps0, double tol) {
    if (c->designs.size() <= 1) return eps <= tol * eps0;
    for (size_t d = 0; d < c->designs.size(); ++d) {
        const double e0 = c->eps0_d[d];
        if (e0 > 0.0 && !(std::sqrt(std::max(c->hpin[16 + d], 0.0)) <= tol * e0)) return false;
    }
    return true;
}

// dot(a, b) of n-vectors into c->scal[slot]
void ddot(feti_ctx* c, int n, const double* a, const double* b, int slot) {
    launch_rowsum_dot(n, 1, a, b, c->part, c->scal + slot, c->st);
    CHECK_LAUNCH();
}

// RHS: d and lambda_0 from the global load f.
void compute_rhs(feti_ctx* c, const double* f) {
    DevTopo& t = c->t;
    hipStream_t st = c->st;
    const Plan& P = c->P;
    if (f != c->f_last) HIPCHK(hipMemcpyAsync(c->f_last, f, sizeof(double) * P.n_dof, hipMemcpyDeviceToDevice, st));
    c->have_f = true;
    launch_scatter_f(t, f, c->fi, c->fbeta, st);
    // g = f_beta - K_beta,i K_ii^{-1} f_i: the two band sweeps, then the coupling rows formed from
    // the element densities (no pass over the stored Z = L^{-1} K_i,beta)
    HIPCHK(hipMemcpyAsync(c->h, c->fi, sizeof(double) * std::max<long long>(1, t.ni_tot), hipMemcpyDeviceToDevice, st));
    launch_bt_fsolve1(t, c->L, c->Li, c->h, st);
    launch_bt_bsolve1(t, c->L, c->Li, c->h, st);
    launch_coupling(t, c->Emod, 1, c->h, c->fbeta, c->g, st);
    launch_local_F(t, c->F64, c->g, c->yb, c->yc, st);
    CHECK_LAUNCH();
    if (P.n_lambda > 0) {
        if (P.method == FETI_DP) {
            launch_fbar(t, c->g, c->yc, c->fbar_s, st);
            if (P.n_cg > 0) {
                launch_coarse(t, 1, 0, c->fbar_s, nullptr, c->Kcc_inv, -1.0, c->vbuf, c->tcbuf, st);
                launch_fold_coarse(t, 1, 0, c->F64, c->vbuf, c->yb, st);
            }
            launch_scatter(t, 1, 0, c->yb, c->d, st);
            HIPCHK(hipMemsetAsync(c->lam0, 0, sizeof(double) * P.n_lambda, st));
        } else {
            launch_scatter(t, 1, 0, c->yb, c->d, st);
            launch_tfeti_e(t, c->fi, c->fbeta, c->Cit, c->e, st);
            launch_small_gemm(c->n_alpha, 1, c->n_alpha, c->GG_inv, c->e, c->tcoef, 1.0, st);
            HIPCHK(hipMemsetAsync(c->lam0, 0, sizeof(double) * P.n_lambda, st));
            launch_proj_apply(t, 1, c->tcoef, c->Rb, -1.0, c->lam0, st);
        }
        CHECK_LAUNCH();
    } else if (P.method == FETI_DP) {
        launch_fbar(t, c->g, c->yc, c->fbar_s, st);
    }
}

// r = P (d - F lam)  (FP64), true residual
void true_residual(feti_ctx* c, const double* lam, double* r) {
    const int n = c->P.n_lambda;
    apply_F(c, 1, FETI_FP64, lam, c->Qtmp);
    launch_axpby(n, 1.0, c->d, 0.0, r, c->st);
    launch_axpby(n, -1.0, c->Qtmp, 1.0, r, c->st);
    project(c, 1, r);
}

void ensure_history(feti_ctx* c, int kd, int need) {
    const int n = c->P.n_lambda;
    if (kd != c->hist_kd) {
        for (double* p : c->hist_chunks) hipFree(p);
        c->hist_chunks.clear();
        c->WH.clear();
        c->QH.clear();
        c->hist_cap = 0;
        c->hist_kd = kd;
    }
    if (need <= c->hist_cap) return;
    int newcap = std::max(need, std::max(16, 2 * c->hist_cap));
    const int add = newcap - c->hist_cap;
    const long long blk = (long long)n * kd;
    double* p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(double) * blk * 2 * add));
    c->hist_chunks.push_back(p);
    for (int i = 0; i < add; ++i) {
        c->WH.push_back(p + blk * (2ll * i));
        c->QH.push_back(p + blk * (2ll * i + 1));
    }
    c->hist_cap = newcap;
    // pointer tables (device): rebuild at full size
    const double** wdev = nullptr;
    const double** qdev = nullptr;
    HIPCHK(hipMalloc(&wdev, sizeof(double*) * newcap));
    HIPCHK(hipMalloc(&qdev, sizeof(double*) * newcap));
    HIPCHK(hipMemcpy(wdev, c->WH.data(), sizeof(double*) * newcap, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(qdev, c->QH.data(), sizeof(double*) * newcap, hipMemcpyHostToDevice));
    if (c->WH_dev) {
        hipStreamSynchronize(c->st);
        hipFree(c->WH_dev);
        hipFree(c->QH_dev);
    }
    c->WH_dev = wdev;
    c->QH_dev = qdev;
    const long long pc = (long long)newcap * kd * kd * (c->segmented ? (long long)c->designs.size() : 1);
    if (pc > c->psi_cap) {
        if (c->Psi) {
            hipStreamSynchronize(c->st);
            hipFree(c->Psi);
        }
        HIPCHK(hipMalloc(&c->Psi, sizeof(double) * pc));
        c->psi_cap = pc;
    }
}

// Deflation of local interface modes (opts.defl_modes; Sec. 6, item (ii)), after the rest of the
// setup: per subdomain F_s = L L^T, B = (omega S~ omega) L, C_s = L^T B, the selected largest
// eigenpairs of C_s, the dual vectors y = diag(w_s) B_s omega^{-1} B x in Y, and the F-orthonormal
// basis of span(Y) in blocks of 64: each block orthogonalised against the kept ones, multiplied by
// F (FP64), F-orthonormalised by the rank-revealing Cholesky of its Gram matrix (Sec. 3.3).
void build_deflation(feti_ctx* c) {
    c->df_nd = c->n_defl = c->n_defl_kept = 0;
    const int m = c->opts.defl_modes;
    const int n = c->P.n_lambda;
    if (m <= 0 || n == 0) return;
    DevTopo& t = c->t;
    hipStream_t st = c->st;
    const int ns = t.n_sub;
    launch_defl_local(t, c->F64, c->Pk, c->bg_w, c->dfOmega, c->dfL, c->dfM, st);
    HIPCHK(hipMemsetAsync(c->info, 0, sizeof(int) * (ns + 8), st));
    launch_potrf(c->d_potrf, ns, t.max_nb, c->dfL, c->info, st);
    CHECK_LAUNCH();
    check_info(c, ns, "deflation: Cholesky of F_s");
    launch_defl_tril(t, c->dfL, st);
    launch_gemm_tn(c->d_df, ns, c->F_tdim, c->dfM, c->dfL, c->dfB, 1.0, 0.0, 0, st);   // B = M^T L = M L
    launch_gemm_tn(c->d_df, ns, c->F_tdim, c->dfL, c->dfB, c->dfC, 1.0, 0.0, 1, st);   // C = L^T B
    launch_defl_eig(t, c->dfC, c->dfB, c->dfOmega, m, c->opts.defl_tau, kDeflGap, kDeflIters, c->dfU, c->dfMu,
                    c->dfCnt, st);
    CHECK_LAUNCH();
    std::vector<int> cnt(ns), col0(ns);
    HIPCHK(hipMemcpyAsync(cnt.data(), c->dfCnt, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int tot = 0;
    for (int s = 0; s < ns; ++s) {
        col0[s] = tot;
        tot += cnt[s];
    }
    c->n_defl = tot;
    if (tot == 0) return;
    HIPCHK(hipMemcpyAsync(c->dfCol0, col0.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    const int nblk = (tot + 63) / 64;
    const long long blk = (long long)n * 64;
    HIPCHK(hipMemsetAsync(c->dfY, 0, sizeof(double) * blk * nblk, st));
    launch_defl_scatter(t, c->bg_w, c->dfU, c->dfCol0, c->dfCnt, c->dfY, st);
    CHECK_LAUNCH();
    const double rr_tol = c->opts.rr_tol > 0 ? c->opts.rr_tol : 1e-12;
    for (int b = 0; b < nblk; ++b) {
        HIPCHK(hipMemcpyAsync(c->Zk, c->dfY + blk * b, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
        if (c->df_nd > 0) {
            launch_gram(n, 64, 64, c->dfQ_dev, c->df_nd, c->Zk, c->part, c->dfPsi, st, false);
            launch_ts_gemm(n, 64, c->df_nd, c->dfW_dev, c->dfPsi, c->Zk, c->Zk, -1.0, 1.0, st, false);
        }
        apply_F(c, 64, FETI_FP64, c->Zk, c->Qk);
        launch_gram(n, 64, 64, c->qk_ptr, 1, c->Zk, c->part, c->Delta, st);
        launch_pivchol(64, c->Delta, rr_tol, c->Tm, c->rank_dev, st, nullptr);
        launch_ts_pair(n, 64, c->zk_ptr, c->qk_ptr, c->Tm, c->dfW[c->df_nd], c->dfQ[c->df_nd], st);
        CHECK_LAUNCH();
        int rank = 0;
        HIPCHK(hipMemcpyAsync(c->hpin, c->rank_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::memcpy(&rank, c->hpin, sizeof(int));
        if (rank > 0) {
            ++c->df_nd;
            c->n_defl_kept += rank;
        }
    }
}

// Z (n_lambda x kd, kd <= 64) <- Z - W_d (Q_d^T Z) against the kept deflation blocks (narrower
// blocks go through the leading columns of a zero 64-column block, so that the 64-wide Gram and
// update kernels serve every width)
void orth_defl(feti_ctx* c, int kd, double* Z) {
    if (c->df_nd == 0) return;
    const int n = c->P.n_lambda;
    hipStream_t st = c->st;
    double* B = Z;
    if (kd != 64) {
        HIPCHK(hipMemsetAsync(c->dfPad, 0, sizeof(double) * n * 64, st));
        launch_pad64(n, kd, 0, Z, c->dfPad, st);
        B = c->dfPad;
    }
    launch_gram(n, 64, 64, c->dfQ_dev, c->df_nd, B, c->part, c->dfPsi, st, false);
    launch_ts_gemm(n, 64, c->df_nd, c->dfW_dev, c->dfPsi, B, B, -1.0, 1.0, st, false);
    if (kd != 64) launch_pad64(n, kd, 1, Z, c->dfPad, st);
    CHECK_LAUNCH();
}

// start correction of a pass: lam += W_d W_d^T r, r -= Q_d W_d^T r (block by block), so that the
// residual is orthogonal to the deflation space
void deflate_start(feti_ctx* c) {
    const int n = c->P.n_lambda;
    for (int b = 0; b < c->df_nd; ++b) {
        launch_gemv_t(n, 64, c->dfW[b], c->r, c->part, c->gam, c->st);
        launch_update_lr(n, 64, c->dfW[b], c->dfQ[b], c->gam, c->lam, c->r, c->st, nullptr);
    }
    CHECK_LAUNCH();
}

struct KrylovOut {
    int iters = 0;
    int reduced = 0;   // iterations that applied the reduced-precision operator
    int kept = 0;
    double eps = 0;
    int status = FETI_OK;
};

// One pass of PCG on the correction: lt accumulates, r is the residual (updated).
// lambda of the current pass: out = lam + lt
void current_iterate(feti_ctx* c, double* out) {
    const int n = c->P.n_lambda;
    HIPCHK(hipMemcpyAsync(out, c->lam, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    launch_axpby(n, 1.0, c->lt, 1.0, out, c->st);
    CHECK_LAUNCH();
}

// Which operator an iteration applies (inexact Krylov: the operator accuracy may be relaxed as
// the residual decreases). A reduced-precision product Q = F_red Z moves the true residual away
// from the recursive one by about eta * |Delta r| <= eta * eps, with eta = |(F_red - F) Z| / |F Z|
// on the iteration's own block: the relative error on the search directions, which grows as they
// concentrate in the low modes of F and can far exceed the error on a generic block. With a
// fixed level (relax > 0) the reduced operator is used once eps <= relax * eps0; otherwise while
// eta * eps <= 0.1 tol eps0, with eta measured by probes (F applied in both precisions, the FP64
// product kept) at the first iteration that passes the test under the prior and every
// kProbeEvery-th reduced iteration after it; the largest measurement is kept.
struct PrecGate {
    static constexpr int kProbeEvery = 16;
    enum { kFp64, kReduced, kProbe };
    int prec = FETI_FP64;
    double sw = 0.0;    // fixed switch level, 0 = measured
    double eta = 0.0;   // prior until the first probe, then the largest measurement
    double tol = 0.0;
    bool measured = false;
    int since = 0;      // reduced iterations since the last probe
    int probes = 0;
    PrecGate(int prec_, double relax, double tol_) : prec(prec_), tol(tol_) {
        if (relax > 0.0)
            sw = relax;
        else
            eta = prec == FETI_BF16X3 ? 1e-3 : 1e-4;
    }
    bool pending = false;   // a probe's norms are not read back yet (one-ahead loop): no reduced product
    int choose(bool replaced, double eps, double eps0) {
        if (prec == FETI_FP64 || replaced) return kFp64;
        if (sw > 0.0) return eps <= sw * eps0 ? kReduced : kFp64;
        if (pending || !(eta * eps <= 0.1 * tol * eps0)) return kFp64;
        if (!measured || since >= kProbeEvery) return kProbe;
        ++since;
        return kReduced;
    }
    void record(double e) {
        eta = measured ? std::max(eta, e) : e;
        measured = true;
        since = 0;
        ++probes;
    }
    // relative error of the FP32 orthogonalisation on probe iterations (opt-in form; reported,
    // not a gate input: see orth_gated)
    double eta_orth = 0.0;
    void record_orth(double e) { eta_orth = std::max(eta_orth, e); }
};

// Q = F Z (k columns) with the operator the gate picks; returns the precision whose product Q holds.
// A probe leaves the FP64 product in Q and records |F_red Z - F Z|_F / |F Z|_F (scratch: n x k).
int gated_apply(feti_ctx* c, PrecGate& g, bool replaced, double eps, double eps0, int k, const double* Z,
                double* Q, double* scratch) {
    const int ch = g.choose(replaced, eps, eps0);
    // the search block's product (Zk -> Qk) replays a captured graph per precision (opts.graphs)
    auto apply = [&](int prec) {
        if (Z == c->Zk && Q == c->Qk && prec >= 0 && prec < 3)
            run_graph(c, c->g_apply[prec], k, [&] { apply_F(c, k, prec, Z, Q); });
        else
            apply_F(c, k, prec, Z, Q);
    };
    if (ch == PrecGate::kFp64) {
        apply(FETI_FP64);
        return FETI_FP64;
    }
    if (ch == PrecGate::kReduced) {
        apply(g.prec);
        return g.prec;
    }
    apply_F(c, k, FETI_FP64, Z, Q);
    apply_F(c, k, g.prec, Z, scratch);
    launch_diff_norms((long long)c->P.n_lambda * k, scratch, Q, c->part, c->scal + 4, c->st);
    CHECK_LAUNCH();
    HIPCHK(hipMemcpyAsync(c->hpin, c->scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    wait_poll(c);
    const double v[2] = {c->hpin[0], c->hpin[1]};
    const double e = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : 0.0;
    g.record(e);
    if (verbose()) fprintf(stderr, "[feti] precision probe: eta %.3e, eps/eps0 %.3e\n", e, eps / eps0);
    return FETI_FP64;
}

KrylovOut run_pcg(feti_ctx* c, PrecGate& g, double eps0, double tol, int max_it, std::vector<double>& hist) {
    KrylovOut o;
    const int n = c->P.n_lambda;
    hipStream_t st = c->st;
    precondition(c, c->r, c->zv, 1, 0);
    HIPCHK(hipMemcpyAsync(c->Zk, c->zv, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    project(c, 1, c->Zk);  // w = P z
    orth_defl(c, 1, c->Zk);
    ddot(c, n, c->r, c->zv, 0);
    launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
    double rz = read_scalars(c);
    o.eps = std::sqrt(std::max(rz, 0.0));
    if (converged(c, o.eps, eps0, tol)) return o;
    bool replaced = false;
    for (int it = 0; it < max_it; ++it) {
        const int p_it = gated_apply(c, g, replaced, o.eps, eps0, 1, c->Zk, c->Qk, c->Qtmp);
        o.reduced += p_it != FETI_FP64;
        ddot(c, n, c->Zk, c->Qk, 1);
        const double wq = read_scalar(c, c->scal + 1);
        if (!(wq > 0.0)) {
            o.status = FETI_EBREAKDOWN;
            break;
        }
        const double a = rz / wq;
        launch_axpby(n, a, c->Zk, 1.0, c->lt, st);
        project(c, 1, c->Qk);
        launch_axpby(n, -a, c->Qk, 1.0, c->r, st);
        precondition(c, c->r, c->zv, 1, 0);
        ddot(c, n, c->r, c->zv, 0);
        launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
        const double rz_new = read_scalars(c);
        o.iters = it + 1;
        o.eps = std::sqrt(std::max(rz_new, 0.0));
        hist.push_back(o.eps);
        if (verbose()) fprintf(stderr, "[feti] pcg it %d prec %d eps/eps0 %.3e\n", it + 1, p_it, o.eps / eps0);
        if (converged(c, o.eps, eps0, tol)) {
            if (o.reduced == 0 || replaced) break;
            // residual replacement after reduced-precision products; PCG restarts from it
            replaced = true;
            current_iterate(c, c->tmpv);
            true_residual(c, c->tmpv, c->r);
            precondition(c, c->r, c->zv, 1, 0);
            ddot(c, n, c->r, c->zv, 0);
            launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
            rz = read_scalars(c);
            o.eps = std::sqrt(std::max(rz, 0.0));
            if (verbose()) fprintf(stderr, "[feti] residual replacement: eps/eps0 %.3e\n", o.eps / eps0);
            if (converged(c, o.eps, eps0, tol)) break;
            HIPCHK(hipMemcpyAsync(c->Zk, c->zv, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            project(c, 1, c->Zk);
            orth_defl(c, 1, c->Zk);
            CHECK_LAUNCH();
            continue;
        }
        const double beta = rz_new / rz;
        rz = rz_new;
        HIPCHK(hipMemcpyAsync(c->Qtmp, c->zv, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        project(c, 1, c->Qtmp);
        orth_defl(c, 1, c->Qtmp);
        launch_axpby(n, 1.0, c->Qtmp, beta, c->Zk, st);
        CHECK_LAUNCH();
    }
    return o;
}

// One pass of Algorithm 1 (simultaneous directions; kd = 1 is full orthogonalisation).
KrylovOut run_sfeti(feti_ctx* c, PrecGate& g, int kd, double eps0, double tol, int max_it,
                    std::vector<double>& hist, std::vector<int>& ranks) {
    // a pass on the reduced-precision operator applies the FP32 preconditioner blocks, if kept
    const int red_pass = g.prec != FETI_FP64;
    KrylovOut o;
    const int n = c->P.n_lambda;
    hipStream_t st = c->st;
    const int one = kd == 1;
    const bool seg = c->segmented && kd == kMaxDirs;
    const bool multi = c->designs.size() > 1 && !c->segmented && kd == c->P.n_groups;
    const int passes = c->opts.reorth == 2 ? 2 : 1;
    // block classical Gram-Schmidt of Z against the stored blocks (per design when segmented),
    // in FP64 or with the FP32 matrix-core forms (64 directions)
    auto orth = [&](int nb_, bool f32, double* Z) {
        for (int pass = 0; pass < passes; ++pass) {
            if (seg) {
                launch_gram_seg(c->t, n, c->QH_dev, nb_, Z, c->part, c->Psi, st, f32);
                launch_ts_seg(c->t, n, nb_, c->WH_dev, c->Psi, (long long)nb_ * 4096, Z, Z, -1.0, 1.0, st, f32);
            } else {
                launch_gram(n, kd, kd, c->QH_dev, nb_, Z, c->part, c->Psi, st, f32);
                launch_ts_gemm(n, kd, nb_, c->WH_dev, c->Psi, Z, Z, -1.0, 1.0, st, f32);
            }
        }
        orth_defl(c, kd, Z);
    };
    // Opt-in (orth_fp32): iterations on the reduced-precision operator also orthogonalise with the
    // FP32 forms. Their error tilts the new block against the stored ones in the F-inner product:
    // a Gram error of u |Q_j| |Z| is a cosine error of about u sqrt(kappa(F)) there, which the
    // later directions cannot remove; on strongly heterogeneous designs that stalls the reduced
    // pass (the caller's FP64 restart then finishes the solve), so FP64 is the default. A probe
    // iteration runs both forms on a copy, keeps the FP64 one and reports |Z_32 - Z_64| / |Z_64|
    // (a Euclidean diagnostic that does not see the F-inner-product amplification).
    const bool orth_red_ok = kd == 64 && c->opts.orth_fp32 && g.prec != FETI_FP64;
    auto orth_gated = [&](int nb_, int p_it, bool probed) {
        if (orth_red_ok && probed) {
            HIPCHK(hipMemcpyAsync(c->Qtmp, c->Zk, sizeof(double) * n * kd, hipMemcpyDeviceToDevice, st));
            orth(nb_, false, c->Zk);
            orth(nb_, true, c->Qtmp);
            launch_diff_norms((long long)n * kd, c->Qtmp, c->Zk, c->part, c->scal + 4, st);
            CHECK_LAUNCH();
            HIPCHK(hipMemcpyAsync(c->hpin, c->scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            wait_poll(c);
            const double e = c->hpin[1] > 0.0 ? std::sqrt(c->hpin[0] / c->hpin[1]) : 0.0;
            g.record_orth(e);
            if (verbose()) fprintf(stderr, "[feti] orthogonalisation probe: eta %.3e\n", e);
        } else {
            orth(nb_, orth_red_ok && p_it != FETI_FP64, c->Zk);
        }
    };
    const double rr_tol = c->opts.rr_tol > 0 ? c->opts.rr_tol : 1e-12;
    precondition(c, c->r, c->Zk, one, red_pass);
    launch_rowsum_dot(n, kd, c->r, c->Zk, c->part, c->scal, st);
    launch_seg_dot(c->t, kd, c->r, c->Zk, c->part, c->scal + 16, st);
    o.eps = std::sqrt(std::max(read_scalars(c), 0.0));
    if (converged(c, o.eps, eps0, tol)) return o;
    project(c, kd, c->Zk);  // W_0 = P Z_0 (in place)
    orth_defl(c, kd, c->Zk);
    // several designs: each stops searching (its direction columns are zeroed) once it has
    // converged or its kept directions span its own dual space, as a single design would
    const int nds = (int)c->designs.size();
    std::vector<unsigned long long> gmask(nds, 0);
    std::vector<int> kept_d(nds, 0);
    unsigned long long all_mask = 0, frozen = 0;
    if (multi)
        for (int d = 0; d < nds; ++d) {
            for (int g = 0; g < c->designs[d].n_groups; ++g) gmask[d] |= 1ull << (c->designs[d].grp0 + g);
            all_mask |= gmask[d];
        }
    if (seg) all_mask = nds >= 64 ? ~0ull : (1ull << nds) - 1;   // bit d: design d
    // the precision gate's eps. Several designs: a reduced product moves design d's true residual
    // away from its recursive one by about eta eps_d, which must stay below 0.1 tol eps0_d for
    // every design still searching; the gate sees the worst ratio eps_d / eps0_d, on the scale
    // of eps0 (one design: eps itself)
    auto gate_eps = [&]() -> double {
        if (nds <= 1) return o.eps;
        double w = 0.0;
        for (int d = 0; d < nds; ++d) {
            const bool fz = multi ? (frozen & gmask[d]) != 0 : seg ? ((frozen >> d) & 1ull) != 0 : false;
            const double e0 = c->eps0_d[d];
            if (fz || !(e0 > 0.0)) continue;
            w = std::max(w, std::sqrt(std::max(c->hpin[16 + d], 0.0)) / e0);
        }
        return w * eps0;
    };
    int nb = 0;
    double best = o.eps;
    int it_best = 0;
    bool replaced = false;
    for (int it = 0; it < max_it && o.kept < n; ++it) {
        ensure_history(c, kd, nb + 1);
        double* Wn = (double*)c->WH[nb];
        double* Qn = (double*)c->QH[nb];
        const int probes_before = g.probes;
        const int p_it = gated_apply(c, g, replaced, gate_eps(), eps0, kd, c->Zk, c->Qk, c->Qtmp);
        const bool probed = g.probes != probes_before;
        o.reduced += p_it != FETI_FP64;
        if (seg) {
            // per design: Delta_d = Q_d^T W_d, its pivoted Cholesky, W, Q, gamma_d = W_d^T r_d
            launch_gram_seg(c->t, n, c->qk_ptr, 1, c->Zk, c->part, c->Delta, st);
            launch_pivchol_seg(nds, c->Delta, rr_tol, c->Tm, reinterpret_cast<int*>(c->scal + 16 + 2 * nds),
                               reinterpret_cast<unsigned long long*>(c->scal + 16 + nds), st);
            launch_ts_pair_seg(c->t, n, c->zk_ptr, c->qk_ptr, c->Tm, Wn, Qn, st);
            launch_gemv_t_seg(c->t, n, Wn, c->r, c->part, c->gam, st);
            launch_update_lr_seg(c->t, n, Wn, Qn, c->gam, c->lt, c->r, st);
        } else {
        // Delta = Q^T W
        launch_gram(n, kd, kd, c->qk_ptr, 1, c->Zk, c->part, c->Delta, st);
        launch_pivchol(kd, c->Delta, rr_tol, c->Tm, c->rank_dev, st,
                       multi ? reinterpret_cast<unsigned long long*>(c->scal + 9) : nullptr);
        launch_ts_pair(n, kd, c->zk_ptr, c->qk_ptr, c->Tm, Wn, Qn, st);
        // gamma = W^T r
        if (kd == 64)
            launch_gemv_t(n, kd, Wn, c->r, c->part, c->gam, st);
        else
            launch_gram(n, kd, 1, c->WH_dev + nb, 1, c->r, c->part, c->gam, st);
        if (c->P.method == FETI_TFETI) {
            launch_update_lr(n, kd, Wn, nullptr, c->gam, c->lt, nullptr, st);
            HIPCHK(hipMemsetAsync(c->tmpv, 0, sizeof(double) * n, st));
            launch_update_lr(n, kd, Qn, nullptr, c->gam, c->tmpv, nullptr, st);
            project(c, 1, c->tmpv);
            launch_axpby(n, -1.0, c->tmpv, 1.0, c->r, st);
        } else {
            launch_update_lr(n, kd, Wn, Qn, c->gam, c->lt, c->r, st);
        }
        }
        CHECK_LAUNCH();
        ++nb;
        run_graph(c, c->g_prec, 2 * kd + red_pass, [&] {
            precondition(c, c->r, c->Zk, one, red_pass);
            launch_rowsum_dot(n, kd, c->r, c->Zk, c->part, c->scal, st);
            launch_seg_dot(c->t, kd, c->r, c->Zk, c->part, c->scal + 16, st);
            project(c, kd, c->Zk);
        });
        orth_gated(nb, p_it, probed);
        CHECK_LAUNCH();
        // eps^2 (scal[0]), the rank (scal[8]) and the per-design values in one copy
        HIPCHK(hipMemcpyAsync(c->hpin, c->scal, (16 + 3 * c->designs.size()) * sizeof(double), hipMemcpyDeviceToHost,
                              st));
        wait_poll(c);
        const double ez = c->hpin[0];
        int rank = 0;
        std::memcpy(&rank, c->hpin + 8, sizeof(int));
        std::vector<int> rank_d(seg ? nds : 0, 0);
        if (seg) {
            std::memcpy(rank_d.data(), c->hpin + 16 + 2 * nds, sizeof(int) * nds);
            rank = 0;
            for (int d = 0; d < nds; ++d) rank += rank_d[d];
        }
        ranks.push_back(rank);
        o.iters = it + 1;
        if (verbose())
            fprintf(stderr, "[feti] sfeti it %d prec %d rank %d eps/eps0 %.3e\n", it + 1, p_it, rank,
                    std::sqrt(std::max(ez, 0.0)) / eps0);
        if (rank == 0) {
            o.status = FETI_EBREAKDOWN;
            break;
        }
        o.kept += rank;
        o.eps = std::sqrt(std::max(ez, 0.0));
        hist.push_back(o.eps);
        if (multi) {
            unsigned long long km = 0;
            std::memcpy(&km, c->hpin + 9, sizeof(km));
            for (int d = 0; d < nds; ++d) {
                if (frozen & gmask[d]) continue;
                kept_d[d] += __builtin_popcountll(km & gmask[d]);
                const bool cd = !(c->eps0_d[d] > 0.0) ||
                                std::sqrt(std::max(c->hpin[16 + d], 0.0)) <= tol * c->eps0_d[d];
                if (cd || kept_d[d] >= c->designs[d].n_lambda) frozen |= gmask[d];
            }
            if (frozen == all_mask && !converged(c, o.eps, eps0, tol)) break;   // every design done
            launch_zero_cols(n, kd, frozen, c->Zk, st);
        } else if (seg) {
            std::vector<unsigned long long> km(nds, 0);
            std::memcpy(km.data(), c->hpin + 16 + nds, sizeof(unsigned long long) * nds);
            for (int d = 0; d < nds; ++d) {
                if ((frozen >> d) & 1ull) continue;
                kept_d[d] += __builtin_popcountll(km[d]);
                const bool cd = !(c->eps0_d[d] > 0.0) ||
                                std::sqrt(std::max(c->hpin[16 + d], 0.0)) <= tol * c->eps0_d[d];
                if (cd || kept_d[d] >= c->designs[d].n_lambda) frozen |= 1ull << d;
            }
            if (frozen == all_mask && !converged(c, o.eps, eps0, tol)) break;   // every design done
            launch_zero_rows(c->t, n, frozen, c->Zk, st);
        }
        const bool conv = converged(c, o.eps, eps0, tol);
        if (o.eps < 0.9 * best) {
            best = o.eps;
            it_best = it;
        }
        // A recurrence on reduced-precision products that diverges or stalls for 10 iterations
        // ends the pass; the caller restarts in FP64 without the stored directions, whose
        // products are then too inexact to orthogonalise against.
        if (!conv && p_it != FETI_FP64 && (o.eps > 1e3 * best || it - it_best > 10)) {
            o.status = FETI_ENOCONV;
            break;
        }
        if (conv && (o.reduced == 0 || replaced)) break;
        if (conv) {
            // The recurrence converged on reduced-precision products: replace the recursive
            // residual by the FP64 one of the current iterate and, if that misses the
            // tolerance, go on in FP64 from it with the stored directions kept.
            replaced = true;
            current_iterate(c, c->tmpv);
            true_residual(c, c->tmpv, c->r);
            precondition(c, c->r, c->Zk, one, red_pass);
            launch_rowsum_dot(n, kd, c->r, c->Zk, c->part, c->scal, st);
            launch_seg_dot(c->t, kd, c->r, c->Zk, c->part, c->scal + 16, st);
            o.eps = std::sqrt(std::max(read_scalars(c), 0.0));
            if (verbose()) fprintf(stderr, "[feti] residual replacement: eps/eps0 %.3e\n", o.eps / eps0);
            if (converged(c, o.eps, eps0, tol)) break;
            project(c, kd, c->Zk);
            orth(nb, false, c->Zk);
            CHECK_LAUNCH();
            best = o.eps;
            it_best = it;
        }
    }
    return o;
}

// Waits for an event by polling (the Krylov loop waits once per iteration).
void wait_event(hipEvent_t e) {
    hipError_t r;
    while ((r = hipEventQuery(e)) == hipErrorNotReady) {
    }
    HIPCHK(r);
}

// Wait until the publish of sequence number seq has reached slot q (launch_publish: the scalars,
// a system-scope fence, then the number). The stream is queried every 1024 polls: once it has
// drained, the number must be there, and its absence is an error rather than an endless wait.
void wait_published(feti_ctx* c, int q, int nsc, long long seq) {
    volatile long long* flag = reinterpret_cast<volatile long long*>(c->hslot[q] + nsc);
    for (long long spins = 1; *flag != seq; ++spins) {
        if ((spins & 1023) == 0) {
            const hipError_t e = hipStreamQuery(c->st);
            if (e == hipSuccess) {
                if (*flag == seq) break;
                throw HipError{"the per-iteration scalars did not reach the host"};
            }
            if (e != hipErrorNotReady) HIPCHK(e);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

// One pass of Algorithm 1 for a single design with the host one iteration behind the device:
// iteration i+1 is enqueued before the scalars of iteration i (eps, rank, a probe's norms) are
// read back, so the device runs the iterations back to back and never waits for the host.
// Iteration i+1 reads the lambda correction of i from one of two buffers and writes its own into
// the other, and stores its directions in the next history slot; when iteration i ends the pass
// (tolerance, rank 0, a stalled reduced recurrence, the dual space exhausted), i+1 is dropped:
// the history count and the correction buffer of i are kept, and every later step (residual
// replacement, the FP64 true residual, recovery) recomputes r and Z from lambda. The precision gate
// chooses from the last eps read back, one iteration older than in the synchronous loop, and
// takes no reduced product while a probe's norms are still on their way.
KrylovOut run_sfeti_ahead(feti_ctx* c, PrecGate& g, int kd, double eps0, double tol, int max_it,
                          std::vector<double>& hist, std::vector<int>& ranks) {
    // a pass on the reduced-precision operator applies the FP32 preconditioner blocks, if kept
    const int red_pass = g.prec != FETI_FP64;
    KrylovOut o;
    const int n = c->P.n_lambda;
    hipStream_t st = c->st;
    const int one = kd == 1;
    const int passes = c->opts.reorth == 2 ? 2 : 1;
    const double rr_tol = c->opts.rr_tol > 0 ? c->opts.rr_tol : 1e-12;
    const size_t nsc = 16 + 3 * c->designs.size();
    auto orth = [&](int nb_) {
        for (int pass = 0; pass < passes; ++pass) {
            launch_gram(n, kd, kd, c->QH_dev, nb_, c->Zk, c->part, c->Psi, st, false);
            launch_ts_gemm(n, kd, nb_, c->WH_dev, c->Psi, c->Zk, c->Zk, -1.0, 1.0, st, false);
        }
        orth_defl(c, kd, c->Zk);
    };
    auto residual_dots = [&] {
        launch_rowsum_dot(n, kd, c->r, c->Zk, c->part, c->scal, st);
        launch_seg_dot(c->t, kd, c->r, c->Zk, c->part, c->scal + 16, st);
    };
    precondition(c, c->r, c->Zk, one, red_pass);
    residual_dots();
    o.eps = std::sqrt(std::max(read_scalars(c), 0.0));
    if (converged(c, o.eps, eps0, tol) || max_it < 1) return o;
    project(c, kd, c->Zk);   // W_0 = P Z_0 (in place)
    orth_defl(c, kd, c->Zk);
    // lambda correction buffers: buf(head) is the output of the last iteration enqueued
    int head = 0;
    auto buf = [&](int i) { return i == 0 ? c->lt : c->lt2; };
    struct Step {
        int p_it = FETI_FP64;
        bool probed = false;
        int out = 0, slot = 0;
        long long seq = 0;
    };
    int nb = 0;
    double eps_seen = o.eps, best = o.eps;
    int it_best = 0;
    bool replaced = false;
    auto enqueue = [&](int it) {
        Step sp;
        ensure_history(c, kd, nb + 1);
        double* Wn = (double*)c->WH[nb];
        double* Qn = (double*)c->QH[nb];
        const int ch = g.choose(replaced, eps_seen, eps0);
        if (ch == PrecGate::kProbe) {
            apply_F(c, kd, FETI_FP64, c->Zk, c->Qk);
            apply_F(c, kd, g.prec, c->Zk, c->Qtmp);
            launch_diff_norms((long long)n * kd, c->Qtmp, c->Qk, c->part, c->scal + 4, st);
            sp.probed = true;
            g.pending = true;
        } else {
            sp.p_it = ch == PrecGate::kReduced ? g.prec : FETI_FP64;
            run_graph(c, c->g_apply[sp.p_it], kd, [&] { apply_F(c, kd, sp.p_it, c->Zk, c->Qk); });
        }
        // Delta = Q^T W, its pivoted Cholesky, W <- W T, Q <- Q T, gamma = W^T r
        launch_gram(n, kd, kd, c->qk_ptr, 1, c->Zk, c->part, c->Delta, st);
        launch_pivchol(kd, c->Delta, rr_tol, c->Tm, c->rank_dev, st, nullptr);
        launch_ts_pair(n, kd, c->zk_ptr, c->qk_ptr, c->Tm, Wn, Qn, st);
        if (kd == 64)
            launch_gemv_t(n, kd, Wn, c->r, c->part, c->gam, st);
        else
            launch_gram(n, kd, 1, c->WH_dev + nb, 1, c->r, c->part, c->gam, st);
        double* lin = buf(head);
        double* lout = buf(1 - head);
        if (c->P.method == FETI_TFETI) {
            launch_update_lr(n, kd, Wn, nullptr, c->gam, lin, nullptr, st, lout);
            HIPCHK(hipMemsetAsync(c->tmpv, 0, sizeof(double) * n, st));
            launch_update_lr(n, kd, Qn, nullptr, c->gam, c->tmpv, nullptr, st);
            project(c, 1, c->tmpv);
            launch_axpby(n, -1.0, c->tmpv, 1.0, c->r, st);
        } else {
            launch_update_lr(n, kd, Wn, Qn, c->gam, lin, c->r, st, lout);
        }
        head = 1 - head;
        sp.out = head;
        ++nb;
        run_graph(c, c->g_prec, 2 * kd + red_pass, [&] {
            precondition(c, c->r, c->Zk, one, red_pass);
            residual_dots();
            project(c, kd, c->Zk);
        });
        orth(nb);
        sp.slot = it & 1;
        sp.seq = ++c->pub_seq;
        launch_publish(c->scal, (int)nsc, c->hslot_dev[sp.slot], sp.seq, st);
        CHECK_LAUNCH();
        return sp;
    };
    Step cur = enqueue(0);
    for (int it = 0;; ++it) {
        Step nxt;
        bool have_nxt = false;
        if (it + 1 < max_it) {
            nxt = enqueue(it + 1);
            have_nxt = true;
        }
        wait_published(c, cur.slot, (int)nsc, cur.seq);
        const double* hs = c->hslot[cur.slot];
        if (cur.probed) {
            const double e = hs[5] > 0.0 ? std::sqrt(hs[4] / hs[5]) : 0.0;
            g.record(e);
            g.pending = false;
            if (verbose()) fprintf(stderr, "[feti] precision probe: eta %.3e\n", e);
        }
        int rank = 0;
        std::memcpy(&rank, hs + 8, sizeof(int));
        const double ez = hs[0];
        ranks.push_back(rank);
        o.iters = it + 1;
        if (verbose())
            fprintf(stderr, "[feti] sfeti it %d prec %d rank %d eps/eps0 %.3e\n", it + 1, cur.p_it, rank,
                    std::sqrt(std::max(ez, 0.0)) / eps0);
        auto drop_next = [&] {
            if (!have_nxt) return;
            --nb;
            head = cur.out;
            if (nxt.probed) g.pending = false;
            have_nxt = false;
        };
        if (rank == 0) {
            o.status = FETI_EBREAKDOWN;
            drop_next();
            break;
        }
        o.reduced += cur.p_it != FETI_FP64;
        o.kept += rank;
        o.eps = std::sqrt(std::max(ez, 0.0));
        eps_seen = o.eps;
        hist.push_back(o.eps);
        const bool conv = converged(c, o.eps, eps0, tol);
        if (o.eps < 0.9 * best) {
            best = o.eps;
            it_best = it;
        }
        if (!conv && cur.p_it != FETI_FP64 && (o.eps > 1e3 * best || it - it_best > 10)) {
            o.status = FETI_ENOCONV;
            drop_next();
            break;
        }
        if ((conv && (o.reduced == 0 || replaced)) || o.kept >= n) {
            drop_next();
            break;
        }
        if (conv) {
            // residual replacement after reduced-precision products (as in the synchronous loop)
            drop_next();
            if (head == 1) {
                std::swap(c->lt, c->lt2);
                head = 0;
            }
            replaced = true;
            current_iterate(c, c->tmpv);
            true_residual(c, c->tmpv, c->r);
            precondition(c, c->r, c->Zk, one, red_pass);
            residual_dots();
            o.eps = std::sqrt(std::max(read_scalars(c), 0.0));
            eps_seen = o.eps;
            if (verbose()) fprintf(stderr, "[feti] residual replacement: eps/eps0 %.3e\n", o.eps / eps0);
            if (converged(c, o.eps, eps0, tol)) break;
            project(c, kd, c->Zk);
            orth(nb);
            CHECK_LAUNCH();
            best = o.eps;
            it_best = it;
            if (it + 1 >= max_it) break;
            nxt = enqueue(it + 1);
            have_nxt = true;
        }
        if (!have_nxt) break;
        cur = nxt;
    }
    // the pass's lambda correction is read from c->lt
    if (head == 1) std::swap(c->lt, c->lt2);
    return o;
}

// recovery of u from lambda (c->lam)
void recover(feti_ctx* c, double* u) {
    DevTopo& t = c->t;
    hipStream_t st = c->st;
    const Plan& P = c->P;
    const double* alpha = nullptr;
    if (P.n_lambda > 0)
        launch_gather_B(t, c->lam, c->xb, st);
    else if (t.nb_tot)
        HIPCHK(hipMemsetAsync(c->xb, 0, sizeof(double) * t.nb_tot, st));
    if (P.method == FETI_DP) {
        if (P.n_cg > 0) {
            if (P.n_lambda > 0) {
                launch_flambda(t, FETI_FP64, 1, c->lam, nullptr, nullptr, c->sw64, c->Ybuf, c->Tbuf, st);
                launch_axpby(t.nc_tot, 1.0, c->fbar_s, 1.0, c->Tbuf, st);
                launch_coarse(t, 1, 0, c->Tbuf, nullptr, c->Kcc_inv, 1.0, c->uc, c->tcbuf, st);
            } else {
                launch_coarse(t, 1, 0, c->fbar_s, nullptr, c->Kcc_inv, 1.0, c->uc, c->tcbuf, st);
            }
        }
        launch_dp_ub(t, c->F64, c->S, c->g, c->xb, c->uc, c->ubeta, c->part, st);
    } else {
        // alpha = (G G^T)^{-1} G (d - F lambda)
        apply_F(c, 1, FETI_FP64, c->lam, c->Qtmp);
        launch_axpby(P.n_lambda, 1.0, c->d, -1.0, c->Qtmp, st);
        launch_proj_G(t, 1, c->Qtmp, c->Rb, c->GY, st);
        launch_small_gemm(c->n_alpha, 1, c->n_alpha, c->GG_inv, c->GY, c->alpha, 1.0, st);
        launch_tfeti_ub(t, c->F64, c->g, c->xb, c->ubeta, c->part, st);
        alpha = c->alpha;
    }
    CHECK_LAUNCH();
    // u_i = K_ii^{-1} (f_i - K_i,beta u_beta): coupling rows from the element densities, then the
    // two band sweeps
    launch_coupling(t, c->Emod, 0, c->ubeta, c->fi, c->ui, st);
    launch_bt_fsolve1(t, c->L, c->Li, c->ui, st);
    launch_bt_bsolve1(t, c->L, c->Li, c->ui, st);
    launch_assemble_loc(t, c->ui, c->ubeta, c->Cit, alpha, c->uloc, st);
    launch_average(t, c->uloc, u, st);
    CHECK_LAUNCH();
}

feti_status do_solve(feti_ctx* c, const double* f, double* u, const double* lam_init, feti_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipEventRecord(c->ev[0], c->st));
    const Plan& P = c->P;
    const int n = P.n_lambda;
    hipStream_t st = c->st;
    compute_rhs(c, f);
    std::vector<double> hist;
    std::vector<int> ranks;
    KrylovOut tot;
    int refinements = 0, fallback = 0, probes = 0;
    double eta_max = 0.0, eta_orth = 0.0;
    double eps0 = 0.0, true_rel = 0.0;
    int status = FETI_OK;
    if (n > 0) {
        // warm start (single design): the multipliers of the last solve, made feasible for this
        // load, lambda_0 + P lambda_prev (TFETI: lambda_0 the minimum-norm solution of G lambda = e,
        // P the projector onto ker G; FETI-DP: lambda_prev itself). The tolerance stays relative to
        // the residual of the cold start lambda_0, so a warm start ends earlier instead of later.
        const bool warm = !lam_init && c->opts.warm_start && c->have_lam && c->designs.size() == 1;
        double eps_cold = 0.0;
        if (warm) {
            HIPCHK(hipMemcpyAsync(c->lam, c->lam0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            true_residual(c, c->lam, c->r);
            precondition(c, c->r, c->zv, 1, 0);
            ddot(c, n, c->r, c->zv, 0);
            launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
            eps_cold = std::sqrt(std::max(read_scalars(c), 0.0));
            HIPCHK(hipMemcpyAsync(c->lam, c->lam_prev, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            project(c, 1, c->lam);
            launch_axpby(n, 1.0, c->lam0, 1.0, c->lam, st);
            CHECK_LAUNCH();
        } else {
            HIPCHK(hipMemcpyAsync(c->lam, lam_init ? lam_init : c->lam0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        }
        true_residual(c, c->lam, c->r);
        const int prec = c->opts.precision;
        const int kd = c->opts.krylov == FETI_SFETI ? P.n_groups : 1;
        // eps0 = sqrt(r0^T z0) with the FP64 preconditioner
        precondition(c, c->r, c->zv, 1, 0);
        ddot(c, n, c->r, c->zv, 0);
        launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
        eps0 = std::sqrt(std::max(read_scalars(c), 0.0));
        if (warm) eps0 = std::max(eps_cold, eps0);
        for (size_t d = 0; d < c->designs.size(); ++d)
            c->eps0_d[d] = c->designs.size() > 1 ? std::sqrt(std::max(c->hpin[16 + d], 0.0)) : eps0;
        hist.push_back(eps0);
        const double tol = c->opts.tol > 0 ? c->opts.tol : 1e-8;
        int max_it = c->opts.max_it > 0 ? c->opts.max_it : n;
        const int max_ref = c->opts.max_refine >= 0 ? c->opts.max_refine : 4;
        // Mixed precision: each pass runs the Krylov iteration with the reduced-precision
        // operator on the current FP64 residual; a pass that breaks down, or whose FP64 true
        // residual does not contract by 10x, hands over to the FP64 operator.
        int cur = prec;
        double prev_rel = 1.0;
        PrecGate gate(prec, c->opts.relax, tol);
        if (eps0 > 0.0) {
            for (int pass = 0;; ++pass) {
                HIPCHK(hipMemsetAsync(c->lt, 0, sizeof(double) * n, st));
                if (c->df_nd > 0) deflate_start(c);
                KrylovOut o;
                const int left = max_it - tot.iters;
                gate.prec = cur;
                if (c->opts.krylov == FETI_PCG)
                    o = run_pcg(c, gate, eps0, tol, left, hist);
                else if (c->designs.size() == 1 && !c->opts.orth_fp32)
                    o = run_sfeti_ahead(c, gate, kd, eps0, tol, left, hist, ranks);
                else
                    o = run_sfeti(c, gate, kd, eps0, tol, left, hist, ranks);
                tot.iters += o.iters;
                tot.reduced += o.reduced;
                tot.kept += o.kept;
                tot.eps = o.eps;
                launch_axpby(n, 1.0, c->lt, 1.0, c->lam, st);
                CHECK_LAUNCH();
                // FP64 true residual
                true_residual(c, c->lam, c->r);
                precondition(c, c->r, c->zv, 1, 0);
                ddot(c, n, c->r, c->zv, 0);
                launch_seg_dot(c->t, 1, c->r, c->zv, c->part, c->scal + 16, st);
                const double et = std::sqrt(std::max(read_scalars(c), 0.0));
                true_rel = et / eps0;
                if (c->designs.size() > 1) {   // the worst design
                    true_rel = 0.0;
                    for (size_t d = 0; d < c->designs.size(); ++d) {
                        c->true_d[d] = std::sqrt(std::max(c->hpin[16 + d], 0.0));
                        if (c->eps0_d[d] > 0.0) true_rel = std::max(true_rel, c->true_d[d] / c->eps0_d[d]);
                    }
                } else {
                    c->true_d[0] = et;
                }
                if (verbose())
                    fprintf(stderr, "[feti] pass %d prec %d iters %d status %d true rel. residual %.3e\n", pass, cur,
                            o.iters, o.status, true_rel);
                if (true_rel <= tol) {
                    status = FETI_OK;
                    break;
                }
                if (tot.iters >= max_it) {
                    status = o.status != FETI_OK ? o.status : FETI_ENOCONV;
                    break;
                }
                if (cur != FETI_FP64) {
                    if (o.status != FETI_OK || !(true_rel < 0.1 * prev_rel) || refinements >= max_ref) {
                        cur = FETI_FP64;
                        ++fallback;
                    }
                } else if (o.status != FETI_OK) {
                    status = o.status;
                    break;
                } else if (pass > max_ref + 1) {
                    status = FETI_ENOCONV;
                    break;
                }
                prev_rel = true_rel;
                ++refinements;
            }
        }
        probes = gate.probes;
        eta_max = gate.measured ? gate.eta : 0.0;
        eta_orth = gate.eta_orth;
    }
    recover(c, u);
    if (n > 0 && (status == FETI_OK || status == FETI_ENOCONV)) {
        HIPCHK(hipMemcpyAsync(c->lam_prev, c->lam, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        c->have_lam = true;
    }
    HIPCHK(hipEventRecord(c->ev[1], st));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->last_ms[3] = ms;
    if (info) {
        info->iters = tot.iters;
        info->refinements = refinements;
        info->status = status;
        info->eps0 = eps0;
        info->eps = tot.eps;
        info->true_rel_res = true_rel;
        info->kept_directions = tot.kept;
        info->fp64_fallback = fallback;
        info->reduced_iters = tot.reduced;
        info->precision_probes = probes;
        info->reduced_rel_err = eta_max;
        info->reduced_orth_err = eta_orth;
        if (info->res_hist && info->res_hist_cap > 0)
            for (int i = 0; i < (int)hist.size() && i < info->res_hist_cap; ++i) info->res_hist[i] = hist[i];
        if (info->rank_hist && info->res_hist_cap > 0)
            for (int i = 0; i < info->res_hist_cap; ++i) info->rank_hist[i] = i < (int)ranks.size() ? ranks[i] : 0;
        info->t_solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status == FETI_ENOCONV) return fail(FETI_ENOCONV, "iteration limit reached before the tolerance");
    if (status == FETI_EBREAKDOWN) return fail(FETI_EBREAKDOWN, "Krylov breakdown: no independent search direction");
    return FETI_OK;
}

feti_status validate_opts(const feti_opts* o) {
    if (!o) return fail(FETI_EINVAL, "null options");
    if (o->scaling != FETI_MULT && o->scaling != FETI_KSCALE) return fail(FETI_EINVAL, "unknown scaling");
    if (o->krylov != FETI_PCG && o->krylov != FETI_FO && o->krylov != FETI_SFETI) return fail(FETI_EINVAL, "unknown krylov");
    if (o->precond != FETI_DIRICHLET && o->precond != FETI_LUMPED && o->precond != FETI_SUPERLUMPED)
        return fail(FETI_EINVAL, "unknown preconditioner");
    if (o->precision != FETI_FP64 && o->precision != FETI_FP32 && o->precision != FETI_BF16X3)
        return fail(FETI_EINVAL, "unknown precision");
    if (!(o->tol >= 0.0)) return fail(FETI_EINVAL, "tol must be >= 0");
    if (o->precond_fp32 != 0 &&
        (o->precond_fp32 != 1 || o->precision == FETI_FP64 || o->krylov == FETI_PCG || o->precond == FETI_SUPERLUMPED))
        return fail(FETI_EINVAL,
                    "precond_fp32 is 0 or 1, and 1 needs a reduced precision, FO or S-FETI and the Dirichlet or "
                    "lumped preconditioner");
    return FETI_OK;
}

template <typename F>
feti_status guarded(F&& fn) {
    try {
        return fn();
    } catch (const HipError& e) {
        return fail(FETI_EHIP, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(FETI_ENOMEM, "host allocation failed");
    } catch (const std::length_error& e) {
        return fail(FETI_ENOMEM, e.what());
    } catch (const std::logic_error& e) {
        return fail(FETI_EINVAL, e.what());
    } catch (const std::runtime_error& e) {
        return fail(FETI_ENOTSPD, e.what());
    }
}

}  // namespace

// ===================================================================================== C ABI
extern "C" {

const char* feti_last_error(void) { return g_err.c_str(); }

feti_status feti_plan_sizes(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts,
                            feti_sizes* out) {
    if (!out) return fail(FETI_EINVAL, "null output");
    try {
        Plan P;
        std::string err = build_plan(mesh, part, opts, P);
        if (!err.empty()) return fail(FETI_EINVAL, err);
        feti_sizes z{};
        z.n_sub = P.n_sub;
        z.n_dof = P.n_dof;
        z.n_el = P.n_el;
        z.n_lambda = P.n_lambda;
        z.n_cg = P.n_cg;
        z.n_alpha = P.n_alpha;
        z.n_groups = P.n_groups;
        z.nb_min = P.n_sub ? *std::min_element(P.n_b.begin(), P.n_b.end()) : 0;
        z.nb_max = P.n_sub ? *std::max_element(P.n_b.begin(), P.n_b.end()) : 0;
        z.n_loc_max = P.n_sub ? *std::max_element(P.n_loc.begin(), P.n_loc.end()) : 0;
        z.n_i_max = P.n_sub ? *std::max_element(P.n_i.begin(), P.n_i.end()) : 0;
        z.band_max = P.n_sub ? *std::max_element(P.band.begin(), P.band.end()) : 0;
        z.sum_nb2 = P.sum_nb2();
        z.sum_nb_nc = P.sum_nb_nc();
        *out = z;
        return FETI_OK;
    } catch (const std::bad_alloc&) {
        return fail(FETI_ENOMEM, "host allocation failed");
    }
}

feti_status feti_adaptive_primal(const feti_mesh* mesh, const feti_partition* part, const double* rho, double p,
                                 double E0, double Emin, double theta, int cap, int* nodes, int nodes_cap,
                                 int* n_out) {
    if (!n_out) return fail(FETI_EINVAL, "null output");
    if (!(theta > 0.0) || cap < 0) return fail(FETI_EINVAL, "need theta > 0 and cap >= 0");
    try {
        std::vector<int> out;
        std::string err = adaptive_primal(mesh, part, rho, p, E0, Emin, theta, cap, out);
        if (!err.empty()) return fail(FETI_EINVAL, err);
        *n_out = (int)out.size();
        if (nodes) {
            if (nodes_cap < (int)out.size()) return fail(FETI_EINVAL, "output capacity too small");
            std::copy(out.begin(), out.end(), nodes);
        }
        return FETI_OK;
    } catch (const std::bad_alloc&) {
        return fail(FETI_ENOMEM, "host allocation failed");
    }
}

feti_status feti_plan_export(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts, int what,
                             int* out, long long cap, long long* n_out) {
    try {
        Plan P;
        std::string err = build_plan(mesh, part, opts, P);
        if (!err.empty()) return fail(FETI_EINVAL, err);
        std::vector<int> v;
        if (what == 0) {
            for (int r = 0; r < P.n_lambda; ++r)
                for (int t = 0; t < 2; ++t) {
                    const int s = P.row_s[2 * r + t];
                    v.push_back(s);
                    v.push_back(s >= 0 ? P.b_loc[P.off_b[s] + P.row_j[2 * r + t]] : -1);
                    v.push_back(P.row_sg[2 * r + t]);
                }
        } else if (what == 1) {
            for (int s = 0; s < P.n_sub; ++s) {
                v.push_back(P.n_loc[s]);
                v.push_back(P.n_i[s]);
                v.push_back(P.n_b[s]);
                v.push_back(P.n_c[s]);
                v.push_back(P.band[s]);
            }
        } else if (what == 2) {
            v = P.corner_dofs;
        } else {
            return fail(FETI_EINVAL, "unknown export");
        }
        if (n_out) *n_out = (long long)v.size();
        if ((long long)v.size() > cap) return fail(FETI_EINVAL, "output capacity too small");
        if (out && !v.empty()) memcpy(out, v.data(), sizeof(int) * v.size());
        return FETI_OK;
    } catch (const std::bad_alloc&) {
        return fail(FETI_ENOMEM, "host allocation failed");
    }
}

feti_status feti_setup(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts, const double* rho,
                       double p, double E0, double Emin, void* stream, feti_ctx** out) {
    if (!out) return fail(FETI_EINVAL, "null output");
    *out = nullptr;
    feti_status vs = validate_opts(opts);
    if (vs != FETI_OK) return vs;
    if (!(p >= 1.0) || !(E0 > 0.0) || !(Emin > 0.0) || !(Emin < E0))
        return fail(FETI_EINVAL, "need p >= 1 and 0 < Emin < E0");
    if (!rho) return fail(FETI_EINVAL, "null density array");
    std::unique_ptr<feti_ctx> c(new feti_ctx());
    std::string err = build_plan(mesh, part, opts, c->P);
    if (!err.empty()) return fail(FETI_EINVAL, err);
    if (opts->krylov == FETI_SFETI && c->P.n_groups > kMaxDirs)
        return fail(FETI_EINVAL, "more than 64 simultaneous directions: set partition.group");
    if (opts->defl_modes < 0 || opts->defl_modes > kDeflMaxModes || !(opts->defl_tau >= 0.0))
        return fail(FETI_EINVAL, "defl_modes must lie in 0..8 and defl_tau be >= 0");
    if (opts->defl_modes > 0 && (opts->method != FETI_DP || opts->recycle))
        return fail(FETI_EINVAL, "deflation of local modes needs FETI-DP without factorisation recycling");
    c->opts = *opts;
    c->p = p;
    c->E0 = E0;
    c->Emin = Emin;
    c->st = (hipStream_t)stream;
    feti_status rs = guarded([&]() -> feti_status {
        build_layout(c.get());
        HIPCHK(hipMemcpyAsync(c->rho, rho, sizeof(double) * c->P.n_el, hipMemcpyDeviceToDevice, c->st));
        numeric_setup(c.get());
        return FETI_OK;
    });
    if (rs != FETI_OK) return rs;
    *out = c.release();
    return FETI_OK;
}

feti_status feti_setup_batched(int n_designs, const feti_mesh* meshes, const feti_partition* parts,
                               const feti_opts* opts, const double* rho, double p, double E0, double Emin,
                               void* stream, feti_ctx** out) {
    if (!out) return fail(FETI_EINVAL, "null output");
    *out = nullptr;
    if (n_designs < 1 || !meshes || !parts) return fail(FETI_EINVAL, "need at least one design");
    feti_status vs = validate_opts(opts);
    if (vs != FETI_OK) return vs;
    if (opts->method != FETI_DP) return fail(FETI_EINVAL, "batched designs need FETI-DP");
    if (opts->defl_modes != 0) return fail(FETI_EINVAL, "deflation of local modes needs a single design");
    if (!(p >= 1.0) || !(E0 > 0.0) || !(Emin > 0.0) || !(Emin < E0))
        return fail(FETI_EINVAL, "need p >= 1 and 0 < Emin < E0");
    if (!rho) return fail(FETI_EINVAL, "null density array");
    std::unique_ptr<feti_ctx> c(new feti_ctx());
    // S-FETI: every design searches along its own direction groups in the same 64 columns
    c->segmented = opts->krylov == FETI_SFETI && n_designs > 1;
    if (c->segmented && n_designs > 64) return fail(FETI_EINVAL, "at most 64 designs per batched S-FETI context");
    std::string err = build_plan_batched(n_designs, meshes, parts, opts, c->P, c->designs, c->segmented);
    if (!err.empty()) return fail(FETI_EINVAL, err);
    if (opts->krylov == FETI_SFETI && c->P.n_groups > kMaxDirs)
        return fail(FETI_EINVAL, "more than 64 simultaneous directions in one design: set partition.group");
    if (c->segmented) c->P.n_groups = kMaxDirs;   // 64 columns; a design's unused ones stay zero
    c->opts = *opts;
    c->p = p;
    c->E0 = E0;
    c->Emin = Emin;
    c->st = (hipStream_t)stream;
    feti_status rs = guarded([&]() -> feti_status {
        build_layout(c.get());
        HIPCHK(hipMemcpyAsync(c->rho, rho, sizeof(double) * c->P.n_el, hipMemcpyDeviceToDevice, c->st));
        numeric_setup(c.get());
        return FETI_OK;
    });
    if (rs != FETI_OK) return rs;
    *out = c.release();
    return FETI_OK;
}

namespace {
// Cache of tuned tile shapes: a JSON object with one entry per line,
//   "key": {"max_red": 32, "max_d": 16, "xcd": 1, "split_d": 4, "fp64_first": 0, "us": 96.5},
std::map<std::string, feti_tuning> read_tune_cache(const char* path) {
    std::map<std::string, feti_tuning> out;
    FILE* f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        const char* q0 = std::strchr(line, '"');
        const char* q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char* br = q1 ? std::strchr(q1, '{') : nullptr;
        if (!br) continue;
        feti_tuning t{};
        if (std::sscanf(br, "{\"max_red\": %d, \"max_d\": %d, \"xcd\": %d, \"split_d\": %d, \"fp64_first\": %d, \"us\": %lf",
                        &t.max_red, &t.max_d, &t.xcd, &t.split_d, &t.fp64_first, &t.us) == 6)
            out[std::string(q0 + 1, q1)] = t;
    }
    std::fclose(f);
    return out;
}

void write_tune_cache(const char* path, const std::map<std::string, feti_tuning>& m) {
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        const feti_tuning& t = kv.second;
        std::fprintf(f,
                     " \"%s\": {\"max_red\": %d, \"max_d\": %d, \"xcd\": %d, \"split_d\": %d, \"fp64_first\": %d, "
                     "\"us\": %.2f}%s\n",
                     kv.first.c_str(), t.max_red, t.max_d, t.xcd, t.split_d, t.fp64_first, t.us,
                     ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
}

// in-solve F*Lambda kernel time (ms, mean over reps after one warm-up) with the current shapes
double time_flambda(feti_ctx* c, int reps) {
    apply_F(c, 64, c->opts.precision, c->Zk, c->Qtmp, true);
    double tot = 0.0;
    for (int r = 0; r < reps; ++r) {
        apply_F(c, 64, c->opts.precision, c->Zk, c->Qtmp, true);
        HIPCHK(hipEventSynchronize(c->ev[3]));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
        tot += ms;
    }
    return tot / std::max(1, reps);
}
}  // namespace

feti_status feti_autotune(feti_ctx* c, int reps, const char* cache_path, feti_tuning* out) {
    if (!c) return fail(FETI_EINVAL, "null context");
    if (c->P.n_lambda == 0) return fail(FETI_EINVAL, "no dual unknowns to tune for");
    return guarded([&]() -> feti_status {
        char key[256];
        std::snprintf(key, sizeof(key), "flambda nsub=%d nb32=%d prec=%d hybrid=%d fp64subs=%d", c->P.n_sub,
                      (c->t.max_nb + 31) / 32, c->opts.precision, c->hybrid ? 1 : 0, c->n_fp64_subs);
        std::map<std::string, feti_tuning> cache = read_tune_cache(cache_path);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            c->tune = hit->second;
            c->tune.from_cache = 1;
            build_fl_tiles(c);
            if (out) *out = c->tune;
            return FETI_OK;
        }
        // Zk, Qtmp: n_lambda x 64 work buffers; their contents do not change the timing
        HIPCHK(hipMemsetAsync(c->Zk, 0, sizeof(double) * c->P.n_lambda * kMaxDirs, c->st));
        const int rp = std::max(1, reps);
        feti_tuning best{2 * kFlWaves, kFlWaves, 1, 4, 0.0, 0.0, 0, 0};
        c->tune = best;
        build_fl_tiles(c);
        const double t_def = time_flambda(c, rp);
        best.us = 1e3 * t_def;
        // the placement of the FP64 tiles (split_d 0, fp64_first) only matters for hybrid lists
        const std::vector<int> sds = c->hybrid ? std::vector<int>{4, 2, 1, 0} : std::vector<int>{4, 2};
        const std::vector<int> ffs = c->hybrid ? std::vector<int>{0, 1} : std::vector<int>{0};
        for (int mr : {32, 16})
            for (int md : {16, 14, 12, 10, 8, 4})
                for (int xc : {1, 0})
                    for (int sd : sds)
                        for (int ff : ffs) {
                            c->tune = feti_tuning{mr, md, xc, sd, 0.0, 0.0, 0, ff};
                            build_fl_tiles(c);
                            const double tm = 1e3 * time_flambda(c, rp);
                            // a change of shapes must gain at least 2% (timing noise keeps the defaults)
                            if (tm < 0.98 * best.us) best = feti_tuning{mr, md, xc, sd, tm, 0.0, 0, ff};
                        }
        best.us_default = 1e3 * t_def;
        c->tune = best;
        build_fl_tiles(c);
        if (cache_path) {
            cache[key] = best;
            write_tune_cache(cache_path, cache);
        }
        if (out) *out = best;
        return FETI_OK;
    });
}

feti_status feti_set_tuning(feti_ctx* c, const feti_tuning* tune) {
    if (!c || !tune) return fail(FETI_EINVAL, "null argument");
    const feti_tuning& q = *tune;
    if (q.max_red < 1 || q.max_red > 2 * kFlWaves || q.max_d < 1 || q.max_d > kFlWaves || q.split_d < 0 ||
        q.split_d > 4 || (q.xcd != 0 && q.xcd != 1) || (q.fp64_first != 0 && q.fp64_first != 1))
        return fail(FETI_EINVAL, "tile shapes out of range");
    return guarded([&]() -> feti_status {
        c->tune = q;
        c->tune.from_cache = 0;
        build_fl_tiles(c);
        return FETI_OK;
    });
}

feti_status feti_design_layout(feti_ctx* c, int d, feti_design* out) {
    if (!c || !out) return fail(FETI_EINVAL, "null argument");
    if (d < 0 || d >= (int)c->designs.size()) return fail(FETI_EINVAL, "design index out of range");
    const DesignMeta& D = c->designs[d];
    out->el0 = D.el0;
    out->n_el = D.n_el;
    out->dof0 = D.dof0;
    out->n_dof = D.n_dof;
    out->sub0 = D.sub0;
    out->n_sub = D.n_sub;
    out->lam0 = D.lam0;
    out->n_lambda = D.n_lambda;
    out->n_groups = D.n_groups;
    return FETI_OK;
}

feti_status feti_design_residuals(feti_ctx* c, double* out, int cap) {
    if (!c || !out) return fail(FETI_EINVAL, "null argument");
    if (cap < (int)c->designs.size()) return fail(FETI_EINVAL, "output smaller than the number of designs");
    for (size_t d = 0; d < c->designs.size(); ++d)
        out[d] = c->eps0_d[d] > 0.0 ? c->true_d[d] / c->eps0_d[d] : 0.0;
    return FETI_OK;
}

feti_status feti_update_rho(feti_ctx* c, const double* rho) {
    if (!c || !rho) return fail(FETI_EINVAL, "null argument");
    return guarded([&]() -> feti_status {
        HIPCHK(hipMemcpyAsync(c->rho, rho, sizeof(double) * c->P.n_el, hipMemcpyDeviceToDevice, c->st));
        numeric_setup(c);
        return FETI_OK;
    });
}

feti_status feti_solve(feti_ctx* c, const double* f, double* u, const double* lambda_init, feti_info* info) {
    if (!c || !f || !u) return fail(FETI_EINVAL, "null argument");
    return guarded([&]() -> feti_status { return do_solve(c, f, u, lambda_init, info); });
}

feti_status feti_compliance_and_grad(feti_ctx* c, const double* rho, const double* f, double* cval, double* dc,
                                     double* u, feti_info* info) {
    if (!c || !cval || !dc) return fail(FETI_EINVAL, "null argument");
    if (!f && !c->have_f) return fail(FETI_EINVAL, "no load given and none stored");
    return guarded([&]() -> feti_status {
        if (rho) {
            HIPCHK(hipMemcpyAsync(c->rho, rho, sizeof(double) * c->P.n_el, hipMemcpyDeviceToDevice, c->st));
            numeric_setup(c);
        }
        double* uu = u ? u : c->u_int;
        feti_status s = do_solve(c, f ? f : c->f_last, uu, nullptr, info);
        if (s != FETI_OK && s != FETI_ENOCONV) return s;
        launch_compliance(c->t, c->f_last, uu, c->rho, c->p, c->E0, c->Emin, c->part, cval, dc, c->st);
        CHECK_LAUNCH();
        return s;
    });
}

feti_status feti_get_lambda(feti_ctx* c, double* lambda) {
    if (!c || !lambda) return fail(FETI_EINVAL, "null argument");
    if (!c->have_lam) return fail(FETI_EINVAL, "no solve has run on this context");
    return guarded([&]() -> feti_status {
        if (c->P.n_lambda > 0)
            HIPCHK(hipMemcpyAsync(lambda, c->lam_prev, sizeof(double) * c->P.n_lambda, hipMemcpyDeviceToDevice,
                                  c->st));
        return FETI_OK;
    });
}

feti_status feti_get_deflation(feti_ctx* c, double* mu, double* Y) {
    if (!c || !mu) return fail(FETI_EINVAL, "null argument");
    if (c->opts.defl_modes <= 0 || !c->dfMu) return fail(FETI_EINVAL, "the context has no deflation");
    return guarded([&]() -> feti_status {
        hipStream_t st = c->st;
        HIPCHK(hipMemcpyAsync(mu, c->dfMu, sizeof(double) * c->t.n_sub * c->opts.defl_modes, hipMemcpyDeviceToDevice,
                              st));
        const long long n = c->P.n_lambda;
        if (Y && c->n_defl > 0)
            for (int b = 0; 64 * b < c->n_defl; ++b) {
                const int w = std::min(64, c->n_defl - 64 * b);
                HIPCHK(hipMemcpy2DAsync(Y + 64 * b, sizeof(double) * c->n_defl, c->dfY + n * 64 * b, sizeof(double) * 64,
                                        sizeof(double) * w, n, hipMemcpyDeviceToDevice, st));
            }
        return FETI_OK;
    });
}

feti_status feti_oc_update(feti_ctx* c, const double* rho, const double* dc, double volfrac, double move, double eta,
                           double rho_min, double* rho_new, double* lagrange) {
    if (!c || !rho || !dc || !rho_new) return fail(FETI_EINVAL, "null argument");
    if (c->designs.size() != 1) return fail(FETI_EINVAL, "the design update takes one design per context");
    if (!(rho_min >= 0.0 && rho_min < 1.0) || !(volfrac > rho_min && volfrac <= 1.0) || !(move > 0.0) || !(eta > 0.0))
        return fail(FETI_EINVAL, "need 0 <= rho_min < volfrac <= 1, move > 0 and eta > 0");
    return guarded([&]() -> feti_status {
        const long long n = c->P.n_el;
        const int nwg = (int)std::min<long long>(1024, std::max<long long>(1, (n + 255) / 256));
        std::vector<double> hp(nwg);
        auto reduce = [&](double lam, int mode) {
            launch_oc_reduce(n, rho, dc, lam, move, eta, rho_min, mode, nwg, c->part, c->st);
            CHECK_LAUNCH();
            HIPCHK(hipMemcpyAsync(hp.data(), c->part, sizeof(double) * nwg, hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            double a = 0.0;
            for (int i = 0; i < nwg; ++i) a = mode == 0 ? a + hp[i] : std::max(a, hp[i]);
            return a;
        };
        const double target = volfrac * (double)n;
        double lo = 0.0, hi = reduce(0.0, 1);
        if (!(hi > 0.0)) hi = 1.0;
        for (int k = 0; k < 200 && reduce(hi, 0) > target; ++k) hi *= 2.0;
        for (int k = 0; k < 200 && hi - lo > 1e-14 * hi; ++k) {
            const double mid = 0.5 * (lo + hi);
            if (reduce(mid, 0) <= target)
                hi = mid;
            else
                lo = mid;
        }
        launch_oc_apply(n, rho, dc, hi, move, eta, rho_min, rho_new, c->st);
        CHECK_LAUNCH();
        if (lagrange) *lagrange = hi;
        return FETI_OK;
    });
}

feti_status feti_destroy(feti_ctx* c) {
    if (!c) return FETI_OK;
    delete c;
    return FETI_OK;
}

feti_status feti_get_sizes(feti_ctx* c, feti_sizes* out) {
    if (!c || !out) return fail(FETI_EINVAL, "null argument");
    const Plan& P = c->P;
    feti_sizes z{};
    z.n_sub = P.n_sub;
    z.n_dof = P.n_dof;
    z.n_el = P.n_el;
    z.n_lambda = P.n_lambda;
    z.n_cg = P.n_cg;
    z.n_alpha = P.n_alpha;
    z.n_groups = P.n_groups;
    z.nb_min = *std::min_element(P.n_b.begin(), P.n_b.end());
    z.nb_max = *std::max_element(P.n_b.begin(), P.n_b.end());
    z.n_loc_max = *std::max_element(P.n_loc.begin(), P.n_loc.end());
    z.n_i_max = *std::max_element(P.n_i.begin(), P.n_i.end());
    z.band_max = *std::max_element(P.band.begin(), P.band.end());
    z.sum_nb2 = P.sum_nb2();
    z.sum_nb_nc = P.sum_nb_nc();
    z.device_bytes = c->bytes;
    z.n_fp64_subs = c->n_fp64_subs;
    z.n_designs = (int)c->designs.size();
    z.n_setup_subs = c->n_setup_subs;
    z.n_defl = c->n_defl;
    z.n_defl_kept = c->n_defl_kept;
    z.sum_nb2_fp64 = 0;
    if (c->hybrid)
        for (int s = 0; s < P.n_sub; ++s)
            if (!c->sub_ok[s]) z.sum_nb2_fp64 += (long long)P.n_b[s] * P.n_b[s];
    *out = z;
    return FETI_OK;
}

feti_status feti_apply_F(feti_ctx* c, int k, int precision, const double* Lambda, double* Q) {
    if (!c || !Lambda || !Q) return fail(FETI_EINVAL, "null argument");
    if (k < 1 || k > kMaxDirs) return fail(FETI_EINVAL, "k must lie in [1, 64]");
    const bool pure = (precision & FETI_PURE) != 0;
    precision &= ~FETI_PURE;
    if (precision != FETI_FP64 && precision != FETI_FP32 && precision != FETI_BF16X3)
        return fail(FETI_EINVAL, "unknown precision");
    return guarded([&]() -> feti_status {
        HIPCHK(hipEventRecord(c->ev[0], c->st));
        apply_F(c, k, precision, Lambda, Q, true, pure);
        HIPCHK(hipEventRecord(c->ev[1], c->st));
        HIPCHK(hipEventSynchronize(c->ev[1]));
        float a = 0, b = 0;
        HIPCHK(hipEventElapsedTime(&a, c->ev[2], c->ev[3]));
        HIPCHK(hipEventElapsedTime(&b, c->ev[0], c->ev[1]));
        c->last_ms[0] = a;
        c->last_ms[1] = b;
        return FETI_OK;
    });
}

feti_status feti_apply_F_noalloc(feti_ctx* c, int k, int precision, const double* Lambda, double* Q) {
    if (!c || !Lambda || !Q) return fail(FETI_EINVAL, "null argument");
    if (k < 1 || k > kMaxDirs) return fail(FETI_EINVAL, "k must lie in [1, 64]");
    const bool pure = (precision & FETI_PURE) != 0;
    precision &= ~FETI_PURE;
    if (precision != FETI_FP64 && precision != FETI_FP32 && precision != FETI_BF16X3)
        return fail(FETI_EINVAL, "unknown precision");
    const long long need = fl_bufs_bytes(c->t, k);
    if (need > kNoAllocScratchBytes)
        return fail(FETI_EINVAL, "feti_apply_F_noalloc: the workspace of this F*Lambda needs " + std::to_string(need) +
                                     " bytes, more than the fixed " + std::to_string(kNoAllocScratchBytes) +
                                     " (use feti_apply_F or fewer columns)");
    if (!c->scratch) return fail(FETI_EHIP, "no-allocation workspace address not set up");
    return guarded([&]() -> feti_status {
        apply_F_with(c, k, precision, Lambda, Q, fl_bufs_in(c->t, k, c->scratch), false, pure);
        return FETI_OK;
    });
}

feti_status feti_apply_precond(feti_ctx* c, const double* r, double* Z, int one_column) {
    if (!c || !r || !Z) return fail(FETI_EINVAL, "null argument");
    const int f32 = (one_column & FETI_PRECOND_FP32) != 0;
    one_column &= ~FETI_PRECOND_FP32;
    if (one_column != 0 && one_column != 1) return fail(FETI_EINVAL, "one_column must be 0 or 1");
    if (f32 && !c->Pk32) return fail(FETI_EINVAL, "FETI_PRECOND_FP32 needs a context set up with precond_fp32 = 1");
    return guarded([&]() -> feti_status {
        precondition(c, r, Z, one_column, f32);
        return FETI_OK;
    });
}

feti_status feti_project(feti_ctx* c, int k, double* Y) {
    if (!c || !Y) return fail(FETI_EINVAL, "null argument");
    if (k < 1 || k > kMaxDirs) return fail(FETI_EINVAL, "k must lie in [1, 64]");
    return guarded([&]() -> feti_status {
        project(c, k, Y);
        return FETI_OK;
    });
}

feti_status feti_rhs(feti_ctx* c, const double* f, double* d, double* lambda0) {
    if (!c || !f) return fail(FETI_EINVAL, "null argument");
    return guarded([&]() -> feti_status {
        compute_rhs(c, f);
        const int n = c->P.n_lambda;
        if (n > 0) {
            if (d) HIPCHK(hipMemcpyAsync(d, c->d, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
            if (lambda0) HIPCHK(hipMemcpyAsync(lambda0, c->lam0, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
        }
        return FETI_OK;
    });
}

feti_status feti_get_local(feti_ctx* c, int s, int what, double* out, long long cap, int* rows, int* cols) {
    if (!c || !out || !rows || !cols) return fail(FETI_EINVAL, "null argument");
    const Plan& P = c->P;
    if (what <= 3 || what == 6)
        if (s < 0 || s >= P.n_sub) return fail(FETI_EINVAL, "subdomain out of range");
    return guarded([&]() -> feti_status {
        HIPCHK(hipStreamSynchronize(c->st));
        std::vector<double> v;
        int nr = 0, nc = 0;
        auto fetch = [&](const double* src, long long n) {
            v.resize(n);
            if (n) HIPCHK(hipMemcpy(v.data(), src, sizeof(double) * n, hipMemcpyDeviceToHost));
        };
        if (what == 0 || what == 2) {
            const SubMeta& M = c->hsubs_act[s];
            std::vector<double> F;
            const long long n = (long long)M.rows_F * M.ldF;
            F.resize(n);
            HIPCHK(hipMemcpy(F.data(), c->F64 + M.off_F, sizeof(double) * n, hipMemcpyDeviceToHost));
            if (what == 0) {
                nr = nc = M.n_b;
                for (int i = 0; i < M.n_b; ++i)
                    for (int j = 0; j < M.n_b; ++j) v.push_back(F[(long long)i * M.ldF + j]);
            } else {
                nr = M.n_b;
                nc = M.n_c;
                for (int j = 0; j < M.n_b; ++j)
                    for (int q = 0; q < M.n_c; ++q) v.push_back(F[(long long)(M.rowT + q) * M.ldF + j]);
            }
        } else if (what == 1) {
            // the packed upper tiles, expanded to the full symmetric n_b x n_b block
            const SubMeta& M = c->hsubs_act[s];
            nr = nc = M.n_b;
            const int nT = (M.n_b + 63) / 64;
            std::vector<double> pk;
            pk.resize((size_t)nT * (nT + 1) / 2 * 4096);
            if (!pk.empty())
                HIPCHK(hipMemcpy(pk.data(), c->Pk + M.off_Pk, sizeof(double) * pk.size(), hipMemcpyDeviceToHost));
            v.assign((size_t)M.n_b * M.n_b, 0.0);
            for (int J = 0; J < nT; ++J)
                for (int I = 0; I <= J; ++I)
                    for (int a = 0; a < 64; ++a)
                        for (int b = 0; b < 64; ++b) {
                            const int row = 64 * I + a, col = 64 * J + b;
                            if (row >= M.n_b || col >= M.n_b) continue;
                            const double e = pk[((size_t)J * (J + 1) / 2 + I) * 4096 + a * 64 + b];
                            v[(size_t)row * M.n_b + col] = e;
                            v[(size_t)col * M.n_b + row] = e;
                        }
        } else if (what == 3) {
            const SubMeta& M = c->hsubs_act[s];
            nr = nc = M.n_c;
            fetch(c->Kc + M.off_Kc, (long long)M.n_c * M.n_c);
        } else if (what == 4) {
            nr = P.n_lambda;
            nc = 2;
            fetch(c->w, 2ll * P.n_lambda);
        } else if (what == 5) {
            // the coarse matrix of design s (its dense diagonal block)
            if (s >= (int)c->designs.size()) throw std::invalid_argument("design index out of range");
            const DesignMeta& D = c->designs[s];
            nr = nc = D.n_cg;
            long long off = 0;
            for (const CoarseBlk& b : c->hcblk)
                if (b.cg0 == D.cg0 && b.n == D.n_cg) off = b.off;
            fetch(c->Kcc + off, (long long)D.n_cg * D.n_cg);
        } else if (what == 6) {
            const SubMeta& M = c->hsubs_act[s];
            nr = M.n_loc;
            nc = 1;
            fetch(c->diag + M.off_loc, M.n_loc);
        } else {
            return fail(FETI_EINVAL, "unknown matrix");
        }
        *rows = nr;
        *cols = nc;
        if ((long long)v.size() > cap) return fail(FETI_EINVAL, "output capacity too small");
        if (!v.empty()) memcpy(out, v.data(), sizeof(double) * v.size());
        return FETI_OK;
    });
}

feti_status feti_last_timing(feti_ctx* c, int what, double* ms) {
    if (!c || !ms || what < 0 || what > 3) return fail(FETI_EINVAL, "bad argument");
    *ms = c->last_ms[what];
    return FETI_OK;
}

}  // extern "C"
