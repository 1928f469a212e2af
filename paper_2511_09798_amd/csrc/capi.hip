// capi.hip -- host runtime and C ABI (include/mqhelm.h) of the MQ-RBF
// Golub-Kahan / Ine-TSVD / HKT solver on one gfx950 GPU.
//
// Every call enqueues its kernels on the problem's stream, keeps all
// Golub-Kahan scalars on the device (no host synchronisation inside the
// loop) and synchronises once before it returns.
#include <float.h>
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "mqhelm.h"

using namespace mqh;

static_assert(MQH_BLOCK_RHS == kBlkRhs, "block size of the lockstep runs");

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? MQH_ENOMEM : MQH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                          \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, #expr);     \
    } while (0)

#define LAUNCHCHK(what)                                       \
    do {                                                      \
        hipError_t _e = hipGetLastError();                    \
        if (_e != hipSuccess) return hip_fail(_e, what);      \
    } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device memory the library holds (every allocation goes through dalloc),
// and an optional cap from the environment variable MQH_DEVICE_MEM_CAP
// (bytes): an allocation that would take the library past the cap fails with
// MQH_ENOMEM before hipMalloc is called.
std::mutex g_mem_mu;
std::unordered_map<void*, size_t> g_mem_sizes;
size_t g_mem_bytes = 0;

int64_t mem_cap() {
    const char* v = getenv("MQH_DEVICE_MEM_CAP");
    if (v == nullptr || *v == '\0') return -1;
    char* end = nullptr;
    const long long c = strtoll(v, &end, 10);
    return (end != v && *end == '\0' && c >= 0) ? (int64_t)c : -1;
}

template <typename T>
int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    const int64_t cap = mem_cap();
    {
        std::lock_guard<std::mutex> lock(g_mem_mu);
        if (cap >= 0 && g_mem_bytes + bytes > (size_t)cap)
            return fail(MQH_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes would take the library "
                                    "past MQH_DEVICE_MEM_CAP = " + std::to_string(cap) + " bytes (" +
                                    std::to_string(g_mem_bytes) + " held)");
        g_mem_bytes += bytes;  // reserved; released below if hipMalloc fails
    }
    hipError_t e = hipMalloc((void**)p, bytes);
    std::lock_guard<std::mutex> lock(g_mem_mu);
    if (e != hipSuccess) {
        *p = nullptr;
        g_mem_bytes -= bytes;
        (void)hipGetLastError();
        return hip_fail(e, "hipMalloc");
    }
    g_mem_sizes[(void*)*p] = bytes;
    return MQH_OK;
}

void dfree_raw(void* p) {
    if (p == nullptr) return;
    {
        std::lock_guard<std::mutex> lock(g_mem_mu);
        auto it = g_mem_sizes.find(p);
        if (it != g_mem_sizes.end()) {
            g_mem_bytes -= it->second;
            g_mem_sizes.erase(it);
        }
    }
    (void)hipFree(p);
}

template <typename T>
void dfree(T*& p) {
    dfree_raw((void*)p);
    p = nullptr;
}

bool all_finite(const double* x, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return false;
    return true;
}

hipMemcpyKind kind_in(uint32_t flags) { return (flags & MQH_FLAG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(uint32_t flags) { return (flags & MQH_FLAG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

// height columns of width bytes, dpitch / spitch bytes apart.  Copies that
// touch host memory go column by column: 2D copies between pageable host
// memory and the device returned wrong data under a kernel tracer on this
// runtime (the first one right, later ones zeros or stale values), while
// plain copies did not.  Device-to-device copies stay 2D.
hipError_t copy_strided(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                     hipMemcpyKind kind, hipStream_t s) {
    if (kind == hipMemcpyDeviceToDevice) return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, kind, s);
    for (size_t c = 0; c < height; ++c) {
        const hipError_t e = hipMemcpyAsync(static_cast<char*>(dst) + c * dpitch,
                                            static_cast<const char*>(src) + c * spitch, width, kind, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Small device-to-host results of a solve, in pinned memory.
struct HostResults {
    GkbState st;
    ParamOut po;
    int32_t svd_status;
    int32_t pad;
};

}  // namespace

// Workspace of the lockstep multi-right-hand-side Golub-Kahan runs: up to
// kBlkRhs runs side by side, run k's arrays at base + k * stride.
struct MultiWs {
    int32_t nz_cap = 0, ell_cap = 0;
    int64_t vstr = 0;     // stride of the length-(ell + 2) arrays (alpha, beta, sv, ftil, y, cvec)
    int64_t bstr = 0;     // stride of a basis, (ell_cap + 1) x ldn
    int64_t gstr = 0;     // stride of the reorthogonalisation partials
    int64_t nstr = 0;     // stride of the norm partials
    double* W = nullptr;  // bases, ldn-padded columns
    double* Z = nullptr;
    double* alpha = nullptr;
    double* beta = nullptr;
    double* sv = nullptr;
    double* ftil = nullptr;
    double* y = nullptr;
    double* cvec = nullptr;
    double* gpart = nullptr;
    double* npart = nullptr;
    double* Vw = nullptr;  // ell_cap x ell_cap per run
    double* V = nullptr;
    GkbState* st = nullptr;
    ParamOut* pout = nullptr;
    int32_t* status = nullptr;
    double* X = nullptr;     // staged right-hand sides, ldn each
    double* Y = nullptr;     // product outputs, ldn each
    double* coef = nullptr;  // coefficients, ldn each
    // block products (FP32-evaluated entries): right-hand sides in the sorted
    // node order, n x kBlkRhs FP32, their split for the FP16 matrix cores
    // (ceil(n / 4) x kBlkRhs quads), the column scales (2^14 for columns of
    // at most unit size; per call for the products of arbitrary vectors),
    // and split-K partials S x kBlkRhs x ldn
    float* Vg = nullptr;
    uint4* Vh = nullptr;
    float* vsc_unit = nullptr;
    float* vsc_data = nullptr;
    double* PB = nullptr;
    int S_rows = 1, S_cols = 1;
    int64_t slice_rows = 0, slice_cols = 0;
    int ft_rows = 2, ft_cols = 2;  // fixed tiles of 16 nodes per wave (blocks of 64 ft fixed nodes)
    // the Golub-Kahan loop of one group as a captured graph, and its key
    hipGraphExec_t graph = nullptr;
    int g_nz = 0;
    int32_t g_ell = 0, g_reorth = -1, g_rs = -1;
};

namespace {
struct BlockCache;  // workspaces of the block calls, kept between calls (defined below)
void block_cache_free(BlockCache* c);
}  // namespace

struct mqh_problem {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t n = 0, n_int = 0, n_bnd = 0, ldn = 0;
    double kappa = 0.0, eps = 1.0;
    int32_t mode = 0;
    bool fixed_shapes = false;
    double center[3] = {0.0, 0.0, 0.0};
    EntryConst ec{};
    // row scaling D = diag(A)^-1 (opt-in): the interior rows' factor, the
    // entry constants of D A, the scaling of the current call's products and
    // the one the stored matrix was assembled with
    double d_int = 1.0;
    EntryConst ec_rs{};
    int32_t rs = 0;
    int32_t A_rs = 0;
    double4* X64 = nullptr;
    float4* X32 = nullptr;
    // FP32-evaluated products: nodes in Morton order within each class (FP32
    // records), perm[q] = original index of sorted node q, one frame centre
    // per block of kMfmFixed sorted nodes, and the weight-folded coefficients
    // of the current product in the sorted order
    float4* XS = nullptr;
    double4* XS64 = nullptr;  // FP64 pair products: sorted coordinates, the product's weights in .w
    int32_t* perm = nullptr;
    int32_t* iperm = nullptr;  // iperm[perm[q]] = q
    float4* frames = nullptr;
    float4* cf = nullptr;
    double blk_tmax = 1.0;  // bound on t = 1 + |P - Q|^2 over node pairs (the block products' entry scale)
    // the single-vector FP32 products over unordered node pairs: work items,
    // their tables, and the row / column partials of a product
    SymLayout sym{};
    int2* sym_items = nullptr;
    int32_t* sym_first = nullptr;
    double* sym_row = nullptr;
    double* sym_col = nullptr;
    // stored matrix: kTile x kTile tiles with the symmetric blocks stored once
    // (layout at the stored operator in op_kernels.hip), its tables, and the
    // product partials (PR per work item, PC per stored tile)
    double* A = nullptr;
    PackedLayout pk{};
    int32_t pk_max_row = 0;
    int64_t pk_tiles = 0;
    int64_t* pk_tile_base = nullptr;
    int4* pk_items = nullptr;
    int32_t* pk_item_first = nullptr;
    double* PR = nullptr;
    double* PC = nullptr;
    // length-ldn vectors (zero past n)
    double* vx = nullptr;
    double* vy = nullptr;
    double* vz = nullptr;
    // Golub-Kahan workspace
    int32_t ell_cap = 0;
    double* W = nullptr;
    double* Z = nullptr;
    double* alpha = nullptr;
    double* beta = nullptr;
    GkbState* st = nullptr;
    double* gpart = nullptr;
    double* cvec = nullptr;
    double* npart = nullptr;
    // projected problem
    double* sv = nullptr;
    double* ftil = nullptr;
    double* Vw = nullptr;
    double* V = nullptr;
    double* y = nullptr;
    ParamOut* pout = nullptr;
    int32_t* svd_status = nullptr;
    double* coef = nullptr;
    HostResults* hres = nullptr;
    // evaluation
    double4* E = nullptr;
    int64_t E_cap = 0;
    double* EP = nullptr;
    int64_t EP_cap = 0;
    double* u = nullptr;
    // learned predictor: features (kMlpIn), outputs (kMlpOut), hidden
    // activations (3 x kMlpWidth), standardisation (2 kMlpIn), FP32
    float* mlp = nullptr;
    ParamOut* pout2 = nullptr;
    // multi-right-hand-side runs
    MultiWs mw;
    BlockCache* bc = nullptr;
    // timing
    hipEvent_t ev[8] = {};
    std::vector<hipEvent_t> pev;
};

namespace {

void to_records(const mqh_problem* p, const double* xyz, int64_t m, double4* r64, float4* r32) {
    for (int64_t i = 0; i < m; ++i) {
        const double x = p->eps * (xyz[3 * i + 0] - p->center[0]);
        const double y = p->eps * (xyz[3 * i + 1] - p->center[1]);
        const double z = p->eps * (xyz[3 * i + 2] - p->center[2]);
        if (r64) r64[i] = make_double4(x, y, z, 0.0);
        if (r32) r32[i] = make_float4((float)x, (float)y, (float)z, 0.0f);
    }
}

// Morton (Z-order) code of a point in a box, 10 bits per axis.
uint32_t spread_bits10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Appends to perm the indices [a, b) of r sorted by Morton code over their
// bounding box (stable, so ties keep the input order).
void morton_order(const std::vector<double4>& r, int64_t a, int64_t b, std::vector<int32_t>& perm) {
    if (b <= a) return;
    double lo[3] = {r[a].x, r[a].y, r[a].z}, hi[3] = {lo[0], lo[1], lo[2]};
    for (int64_t i = a; i < b; ++i) {
        const double v[3] = {r[i].x, r[i].y, r[i].z};
        for (int d = 0; d < 3; ++d) {
            lo[d] = v[d] < lo[d] ? v[d] : lo[d];
            hi[d] = v[d] > hi[d] ? v[d] : hi[d];
        }
    }
    double ext = hi[0] - lo[0];
    for (int d = 1; d < 3; ++d) ext = hi[d] - lo[d] > ext ? hi[d] - lo[d] : ext;
    const double scale = ext > 0.0 ? 1024.0 / ext : 0.0;
    std::vector<std::pair<uint32_t, int32_t>> key((size_t)(b - a));
    for (int64_t i = a; i < b; ++i) {
        const double v[3] = {r[i].x, r[i].y, r[i].z};
        uint32_t code = 0;
        for (int d = 0; d < 3; ++d) {
            double s = (v[d] - lo[d]) * scale;
            s = s < 0.0 ? 0.0 : (s > 1023.0 ? 1023.0 : s);
            code |= spread_bits10((uint32_t)s) << d;
        }
        key[(size_t)(i - a)] = {code, (int32_t)i};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint32_t, int32_t>& u, const std::pair<uint32_t, int32_t>& v) {
                         return u.first < v.first;
                     });
    for (const auto& k : key) perm.push_back(k.second);
}

// Sorted records and one frame centre (bounding-box midpoint) per block of
// kMfmFixed sorted nodes, interior blocks first.
void sorted_layout(const std::vector<double4>& r, int64_t n, int64_t n_int, std::vector<int32_t>& perm,
                   std::vector<float4>& rs32, std::vector<float4>& frames, std::vector<double4>* rs64 = nullptr) {
    perm.clear();
    perm.reserve((size_t)n);
    morton_order(r, 0, n_int, perm);
    morton_order(r, n_int, n, perm);
    std::vector<double4> rs((size_t)n);
    rs32.resize((size_t)n);
    for (int64_t q = 0; q < n; ++q) {
        rs[(size_t)q] = r[(size_t)perm[(size_t)q]];
        rs32[(size_t)q] = make_float4((float)rs[(size_t)q].x, (float)rs[(size_t)q].y, (float)rs[(size_t)q].z, 0.0f);
    }
    const int64_t nb_int = (n_int + kMfmFixed - 1) / kMfmFixed;
    const int64_t nb = mfm_blocks(n, n_int);
    frames.assign((size_t)nb, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
    for (int64_t b = 0; b < nb; ++b) {
        const bool fint = b < nb_int;
        const int64_t f0 = fint ? b * kMfmFixed : n_int + (b - nb_int) * kMfmFixed;
        const int64_t fe = fint ? n_int : n;
        const int64_t f1 = f0 + kMfmFixed < fe ? f0 + kMfmFixed : fe;
        double lo[3] = {rs[f0].x, rs[f0].y, rs[f0].z}, hi[3] = {lo[0], lo[1], lo[2]};
        for (int64_t i = f0; i < f1; ++i) {
            const double v[3] = {rs[i].x, rs[i].y, rs[i].z};
            for (int d = 0; d < 3; ++d) {
                lo[d] = v[d] < lo[d] ? v[d] : lo[d];
                hi[d] = v[d] > hi[d] ? v[d] : hi[d];
            }
        }
        frames[(size_t)b] = make_float4((float)(0.5 * (lo[0] + hi[0])), (float)(0.5 * (lo[1] + hi[1])),
                                        (float)(0.5 * (lo[2] + hi[2])), 0.0f);
    }
    if (rs64 != nullptr) rs64->swap(rs);
}

// Tables of the tiled stored matrix: tile rows (interior tiles first), the
// first stored tile of each, and the work items of a product (at most
// kTileChunk consecutive tiles of one tile row).
struct PackedTables {
    int32_t nti = 0, nt = 0, max_row = 0;
    std::vector<int64_t> tile_base;
    std::vector<int4> items;
    std::vector<int32_t> item_first;
};

void packed_tables(int64_t n, int64_t n_int, PackedTables& t) {
    t.nti = (int32_t)((n_int + kTile - 1) / kTile);
    t.nt = t.nti + (int32_t)((n - n_int + kTile - 1) / kTile);
    t.tile_base.assign((size_t)t.nt + 1, 0);
    t.item_first.assign((size_t)t.nt + 1, 0);
    t.items.clear();
    t.max_row = 0;
    for (int32_t R = 0; R < t.nt; ++R) {
        const int32_t ntr = R < t.nti ? t.nt - R : t.nti + (t.nt - R);
        t.max_row = ntr > t.max_row ? ntr : t.max_row;
        t.tile_base[(size_t)R + 1] = t.tile_base[(size_t)R] + ntr;
        t.item_first[(size_t)R] = (int32_t)t.items.size();
        for (int32_t p0 = 0; p0 < ntr; p0 += kTileChunk)
            t.items.push_back(make_int4(R, p0, ntr - p0 < kTileChunk ? ntr - p0 : kTileChunk, 0));
    }
    t.item_first[(size_t)t.nt] = (int32_t)t.items.size();
}

// Entry constants of the operator the current call runs on: A, or D A with
// D = diag(A)^-1.  The scaling only changes the interior rows' constants
// (kappa^2, eps^2, 2 eps^2 times 1 / (3 eps^2 + kappa^2)): boundary rows have
// A_ii = phi(0) = 1.
const EntryConst& op_ec(const mqh_problem* p) { return p->rs ? p->ec_rs : p->ec; }

// Select the row scaling of the call's products (0: A, 1: D A); a stored
// matrix assembled for the other scaling is assembled again.
int set_row_scale(mqh_problem* p, int32_t rs) {
    if (rs != 0 && rs != 1) return fail(MQH_EINVAL, "row_scale must be 0 or 1");
    p->rs = rs;
    if (p->mode == MQH_OP_STORED_FP64 && p->A_rs != rs) {
        launch_assemble_packed(p->X64, p->pk, p->pk_max_row, op_ec(p), p->A, p->stream);
        LAUNCHCHK("assembly");
        p->A_rs = rs;
    }
    return MQH_OK;
}

// Right-hand sides to D f: the interior entries of nz staged vectors
// (stride apart) times 1 / (3 eps^2 + kappa^2), when the call scales rows.
int scale_rhs(mqh_problem* p, double* x, int nz, int64_t stride) {
    if (p->rs == 0) return MQH_OK;
    launch_scale(x, p->n_int, p->d_int, nz, stride, p->stream);
    LAUNCHCHK("row scaling of the data");
    return MQH_OK;
}

// One product y = op(A) x - shift z on device vectors (x, z of length ldn,
// zero-padded).  shift from *shift_ptr when non-null.
// Work items of the pair products (SymLayout): blocks of kMfmFixed sorted
// nodes per class; super-rows of F fixed blocks and segments of Lb loop
// blocks, the largest (F, Lb) that still gives enough items to fill the GPU;
// first[k] indexes the items in (super-row, segment) order, the list itself
// is in launch order.
void sym_tables(int64_t n, int64_t n_int, SymLayout& L, std::vector<int2>& items, std::vector<int32_t>& first) {
    L = SymLayout{};
    L.n = n;
    L.n_int = n_int;
    L.nb_int = (int32_t)((n_int + kMfmFixed - 1) / kMfmFixed);
    L.nb = L.nb_int + (int32_t)((n - n_int + kMfmFixed - 1) / kMfmFixed);
    static const int shapes[][2] = {{8, 14}, {4, 8}, {2, 4}, {1, 2}};
    for (const auto& sh : shapes) {
        items.clear();
        first.clear();
        const int F = sh[0], Lb = sh[1];
        const int nsr = (L.nb + F - 1) / F;
        for (int k = 0; k < nsr; ++k) {
            first.push_back((int32_t)items.size());
            const int nseg = (L.nb - k * F + Lb - 1) / Lb;
            for (int sg = 0; sg < nseg; ++sg) items.push_back(make_int2(k, sg));
        }
        first.push_back((int32_t)items.size());
        L.F = F;
        L.Lb = Lb;
        L.nsr = nsr;
        L.nitems = (int32_t)items.size();
        if (L.nitems >= 1200) break;
    }
    // launch order: items by their number of block pairs, largest first
    // (stable), so the last workgroups to start are the short ones
    auto pairs = [&](const int2& it) {
        const int b0 = it.x * L.F, b1 = std::min(b0 + L.F, L.nb);
        const int c0 = b0 + it.y * L.Lb, c1 = std::min(c0 + L.Lb, L.nb);
        int64_t cnt = 0;
        for (int b = b0; b < b1; ++b) cnt += std::max(0, c1 - std::max(c0, b));
        return cnt;
    };
    std::stable_sort(items.begin(), items.end(), [&](const int2& a, const int2& b) { return pairs(a) > pairs(b); });
}

int op_product(mqh_problem* p, int trans, const double* x, const double* shift_ptr, double shift_val, const double* z,
               double* y, const GkbState* st, bool timed) {
    hipStream_t s = p->stream;
    if (p->mode == MQH_OP_MATFREE_FP32) {
        // x into the sorted node order, folded into the entry coefficients
        // (outside the timed span)
        launch_gather_coef(x, p->perm, p->n, op_ec(p), p->cf, st, s);
        LAUNCHCHK("gather");
    } else if (p->mode == MQH_OP_MATFREE_FP64) {
        launch_gather_w64(x, p->perm, p->n, p->XS64, st, s);
        LAUNCHCHK("gather");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        size_t k = p->pev.size();
        for (int q = 0; q < 2; ++q) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            p->pev.push_back(ev);
        }
        e0 = p->pev[k];
        e1 = p->pev[k + 1];
        HIPCHK(hipEventRecord(e0, s));
    }
    if (p->mode == MQH_OP_STORED_FP64) {
        launch_packed_product(trans, p->A, p->pk, x, p->PR, p->PC, st, s);
        LAUNCHCHK("stored product");
        if (timed) HIPCHK(hipEventRecord(e1, s));
        launch_packed_reduce(trans, p->pk, p->PR, p->PC, shift_ptr, shift_val, z, y, st, s);
        LAUNCHCHK("stored product reduction");
        return MQH_OK;
    }
    if (p->mode == MQH_OP_MATFREE_FP32) {
        launch_mfs_product(trans, p->XS, p->frames, p->cf, p->sym, op_ec(p), p->sym_row, p->sym_col, st, s);
        LAUNCHCHK("pair product");
        if (timed) HIPCHK(hipEventRecord(e1, s));
        launch_mfs_reduce(p->sym, p->sym_row, p->sym_col, p->perm, shift_ptr, shift_val, z, y, st, s);
        LAUNCHCHK("pair product reduction");
        return MQH_OK;
    }
    // FP64 matrix-free: the same pair structure with FP64 entries
    launch_mfs64_product(trans, p->XS64, p->sym, op_ec(p), p->sym_row, p->sym_col, st, s);
    LAUNCHCHK("FP64 pair product");
    if (timed) HIPCHK(hipEventRecord(e1, s));
    launch_mfs_reduce(p->sym, p->sym_row, p->sym_col, p->perm, shift_ptr, shift_val, z, y, st, s);
    LAUNCHCHK("pair product reduction");
    return MQH_OK;
}

int ensure_gkb(mqh_problem* p, int32_t ell) {
    if (ell <= p->ell_cap) return MQH_OK;
    dfree(p->W);
    dfree(p->Z);
    dfree(p->alpha);
    dfree(p->beta);
    dfree(p->gpart);
    dfree(p->cvec);
    dfree(p->sv);
    dfree(p->ftil);
    dfree(p->Vw);
    dfree(p->V);
    dfree(p->y);
    p->ell_cap = 0;
    const int64_t cols = (int64_t)ell + 1;
    int rc;
    if ((rc = dalloc(&p->W, (size_t)(cols * p->ldn)))) return rc;
    if ((rc = dalloc(&p->Z, (size_t)(cols * p->ldn)))) return rc;
    HIPCHK(hipMemsetAsync(p->W, 0, (size_t)(cols * p->ldn) * sizeof(double), p->stream));
    HIPCHK(hipMemsetAsync(p->Z, 0, (size_t)(cols * p->ldn) * sizeof(double), p->stream));
    if ((rc = dalloc(&p->alpha, (size_t)cols))) return rc;
    if ((rc = dalloc(&p->beta, (size_t)cols + 1))) return rc;
    if ((rc = dalloc(&p->gpart, (size_t)cgs_partial_doubles(p->n, cols)))) return rc;
    if ((rc = dalloc(&p->cvec, (size_t)cols))) return rc;
    if ((rc = dalloc(&p->sv, (size_t)cols))) return rc;
    if ((rc = dalloc(&p->ftil, (size_t)cols + 1))) return rc;
    if ((rc = dalloc(&p->Vw, svd_ws_doubles(ell)))) return rc;
    if ((rc = dalloc(&p->V, (size_t)ell * (size_t)ell))) return rc;
    if ((rc = dalloc(&p->y, (size_t)cols))) return rc;
    p->ell_cap = ell;
    return MQH_OK;
}

// f must be staged in p->vx.  Runs Algorithm 1 with ell steps; everything stays on the device.
// Golub-Kahan steps [j0, j1) of a run of at most ell steps (j1 < 0: ell);
// j0 = 0 starts the run from p->vx (beta_1 w_1 = f).  Steps after a
// breakdown are no-ops on the device, so a run may be enqueued in pieces.
int run_gkb(mqh_problem* p, int32_t ell, int32_t reorth, bool timed, int32_t j0 = 0, int32_t j1 = -1) {
    hipStream_t s = p->stream;
    const int64_t n = p->n, ldn = p->ldn;
    const int nbq = sumsq_blocks(n);
    const int nbu = update_blocks(n);
    if (j1 < 0) j1 = ell;
    if (j0 == 0) {
        launch_init_state(p->st, ell, p->alpha, p->beta, s);
        LAUNCHCHK("init state");
        launch_sumsq_partial(p->vx, n, p->npart, nbq, p->st, s);
        launch_finalize_scale(p->npart, nbq, 0, 0, n, p->alpha, p->beta, p->st, p->vx, p->W, s);
        LAUNCHCHK("initial normalisation");
    }
    auto orthonormalize = [&](double* v, const double* V, int32_t m, int kind, int32_t j, double* dst) -> int {
        int nparts;
        if (reorth && m > 0) {
            launch_gemvt(V, ldn, n, m, v, p->gpart, p->cvec, p->st, s);
            if (m <= kFusedCgsMaxCols) {
                launch_update_gemvt(V, ldn, n, m, p->cvec, v, p->gpart, p->st, s);
            } else {
                launch_update(V, ldn, n, m, p->cvec, v, nullptr, p->st, s);
                launch_gemvt(V, ldn, n, m, v, p->gpart, p->cvec, p->st, s);
            }
            launch_update(V, ldn, n, m, p->cvec, v, p->npart, p->st, s);
            nparts = nbu;
        } else {
            launch_sumsq_partial(v, n, p->npart, nbq, p->st, s);
            nparts = nbq;
        }
        launch_finalize_scale(p->npart, nparts, kind, j, n, p->alpha, p->beta, p->st, v, dst, s);
        LAUNCHCHK("reorthogonalisation / normalisation");
        return MQH_OK;
    };
    int rc;
    for (int32_t j = j0; j < j1; ++j) {
        double* Wj = p->W + (int64_t)j * ldn;
        double* Zj = p->Z + (int64_t)j * ldn;
        // r = A^T w_j - beta_j z_{j-1}
        if ((rc = op_product(p, 1, Wj, p->beta + j, 0.0, j > 0 ? p->Z + (int64_t)(j - 1) * ldn : nullptr, p->vy,
                             p->st, timed)))
            return rc;
        if ((rc = orthonormalize(p->vy, p->Z, j, 1, j, Zj))) return rc;
        // p = A z_j - alpha_j w_j
        if ((rc = op_product(p, 0, Zj, p->alpha + j, 0.0, Wj, p->vy, p->st, timed))) return rc;
        if ((rc = orthonormalize(p->vy, p->W, j + 1, 2, j, p->W + (int64_t)(j + 1) * ldn))) return rc;
    }
    return MQH_OK;
}

// ---------------------------------------------------------------------------
// Lockstep multi-right-hand-side Golub-Kahan runs: up to kBlkRhs independent
// runs of Algorithm 1 on the same A, step j of every run enqueued together so
// that each pass over A serves all of them (a block product with the
// FP32-evaluated entries; one product per run for the FP64 forms).  Each run
// keeps its own scalars, bases and breakdown state, exactly as a single run.
// ---------------------------------------------------------------------------

void multi_free(MultiWs& w) {
    if (w.graph != nullptr) (void)hipGraphExecDestroy(w.graph);
    w.graph = nullptr;
    w.g_nz = 0;
    w.g_reorth = -1;
    dfree(w.W);
    dfree(w.Z);
    dfree(w.alpha);
    dfree(w.beta);
    dfree(w.sv);
    dfree(w.ftil);
    dfree(w.y);
    dfree(w.cvec);
    dfree(w.gpart);
    dfree(w.npart);
    dfree(w.Vw);
    dfree(w.V);
    dfree(w.st);
    dfree(w.pout);
    dfree(w.status);
    dfree(w.X);
    dfree(w.Y);
    dfree(w.coef);
    dfree(w.Vg);
    dfree(w.Vh);
    dfree(w.vsc_unit);
    dfree(w.vsc_data);
    dfree(w.PB);
    w.nz_cap = 0;
    w.ell_cap = 0;
}

// Slice count S and length (whole LDS chunks) of a block product aiming at
// target_blocks workgroups.
void block_slices(const mqh_problem* p, int ft, int64_t target_blocks, int& S, int64_t& len) {
    const int64_t n = p->n, nb = mfh_block_blocks(n, p->n_int, ft);
    int64_t s = (target_blocks + nb - 1) / nb;
    if (s < 1) s = 1;
    if (s > kMaxSlices) s = kMaxSlices;
    int64_t l = (n + s - 1) / s;
    l = round_up(l < kMfmChunk ? kMfmChunk : l, kMfmChunk);
    s = (n + l - 1) / l;
    S = (int)(s < 1 ? 1 : s);
    len = l;
}

// Heuristic shapes: a few rounds of resident workgroups over the chip.
void block_shapes(mqh_problem* p, MultiWs& w) {
    w.ft_rows = w.ft_cols = 2;
    block_slices(p, 2, 4096, w.S_rows, w.slice_rows);
    w.S_cols = w.S_rows;
    w.slice_cols = w.slice_rows;
}

// Autotuner of the block products: the tile shape (64 or 128 fixed nodes
// per workgroup, one or two 16-node tiles per wave) and the split of the
// loop range (candidates aiming at 1024 .. 16384 workgroups, about one to
// sixteen rounds of resident workgroups).  Each candidate is timed as the
// whole product (the slice kernel and the reduction of its nz-column
// partials) on a pseudo-random operand, once untimed and then five times
// between event pairs on the problem's stream; the best of the five
// decides, per direction.  w.PB must hold kMaxSlices slices.
int tune_block_shapes(mqh_problem* p, MultiWs& w, int nz) {
    hipStream_t s = p->stream;
    launch_fill_hash(w.Vg, p->n * kBlkRhs, s);
    launch_split_block(w.Vg, p->n, w.vsc_unit, w.Vh, s);
    LAUNCHCHK("tuning operand");
    const BlockEntry be = block_entry(op_ec(p), p->blk_tmax);
    struct Cand {
        int ft, S;
        int64_t len;
    };
    std::vector<Cand> cand;
    for (int ft = 1; ft <= 2; ++ft)
        for (int64_t target = 1024; target <= 16384; target *= 2) {
            int S;
            int64_t len;
            block_slices(p, ft, target, S, len);
            bool seen = false;
            for (auto& c : cand) seen = seen || (c.ft == ft && c.S == S);
            if (!seen) cand.push_back(Cand{ft, S, len});
        }
    constexpr int kReps = 5;
    hipEvent_t ev[kReps + 1] = {};
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    int rc = MQH_OK;
    auto product = [&](int trans, const Cand& c) {
        launch_mfh_block(trans, c.ft, p->XS, p->frames, w.Vh, w.vsc_unit, p->n, p->n_int, c.S, c.len, be, w.PB,
                         p->ldn, s);
        launch_reduce_block(w.PB, p->ldn, c.S, p->n, nz, p->perm, nullptr, 0, nullptr, 0, w.Y, p->ldn, nullptr, s);
    };
    for (int trans = 0; trans < 2 && rc == MQH_OK; ++trans) {
        float best = 0.f;
        for (auto& c : cand) {
            product(trans, c);
            hipError_t e = hipEventRecord(ev[0], s);
            for (int r = 0; r < kReps && e == hipSuccess; ++r) {
                product(trans, c);
                e = hipGetLastError();
                if (e == hipSuccess) e = hipEventRecord(ev[r + 1], s);
            }
            if (e == hipSuccess) e = hipEventSynchronize(ev[kReps]);
            float t = 0.f;
            for (int r = 0; r < kReps && e == hipSuccess; ++r) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
                if (r == 0 || ms < t) t = ms;
            }
            if (e != hipSuccess) {
                rc = hip_fail(e, "block-product tuning");
                break;
            }
            if (best == 0.f || t < best) {
                best = t;
                (trans ? w.ft_cols : w.ft_rows) = c.ft;
                (trans ? w.S_cols : w.S_rows) = c.S;
                (trans ? w.slice_cols : w.slice_rows) = c.len;
            }
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
}

int ensure_multi(mqh_problem* p, int nz, int32_t ell) {
    MultiWs& w = p->mw;
    if (nz <= w.nz_cap && ell <= w.ell_cap) return MQH_OK;
    const int zc = nz > w.nz_cap ? nz : w.nz_cap;
    const int32_t lc = ell > w.ell_cap ? ell : w.ell_cap;
    multi_free(w);
    const int64_t n = p->n, ldn = p->ldn, cols = (int64_t)lc + 1;
    w.vstr = (int64_t)lc + 2;
    w.bstr = cols * ldn;
    w.gstr = cgs_partial_doubles(n, cols);
    w.nstr = update_blocks(n) > 1024 ? update_blocks(n) : 1024;
    const size_t Z = (size_t)zc;
    int rc;
    if ((rc = dalloc(&w.W, Z * (size_t)w.bstr)) || (rc = dalloc(&w.Z, Z * (size_t)w.bstr)) ||
        (rc = dalloc(&w.alpha, Z * (size_t)w.vstr)) || (rc = dalloc(&w.beta, Z * (size_t)w.vstr)) ||
        (rc = dalloc(&w.sv, Z * (size_t)w.vstr)) || (rc = dalloc(&w.ftil, Z * (size_t)w.vstr)) ||
        (rc = dalloc(&w.y, Z * (size_t)w.vstr)) || (rc = dalloc(&w.cvec, Z * (size_t)w.vstr)) ||
        (rc = dalloc(&w.gpart, Z * (size_t)w.gstr)) || (rc = dalloc(&w.npart, Z * (size_t)w.nstr)) ||
        (rc = dalloc(&w.Vw, Z * svd_ws_doubles(lc))) || (rc = dalloc(&w.V, Z * (size_t)lc * (size_t)lc)) ||
        (rc = dalloc(&w.st, Z)) || (rc = dalloc(&w.pout, Z)) || (rc = dalloc(&w.status, Z)) ||
        (rc = dalloc(&w.X, Z * (size_t)ldn)) || (rc = dalloc(&w.Y, Z * (size_t)ldn)) ||
        (rc = dalloc(&w.coef, Z * (size_t)ldn))) {
        multi_free(w);
        return rc;
    }
    hipStream_t s = p->stream;
    // zero padding past n and unused basis columns
    hipError_t e;
    if ((e = hipMemsetAsync(w.W, 0, Z * (size_t)w.bstr * sizeof(double), s)) ||
        (e = hipMemsetAsync(w.Z, 0, Z * (size_t)w.bstr * sizeof(double), s)) ||
        (e = hipMemsetAsync(w.X, 0, Z * (size_t)ldn * sizeof(double), s)) ||
        (e = hipMemsetAsync(w.Y, 0, Z * (size_t)ldn * sizeof(double), s))) {
        multi_free(w);
        return hip_fail(e, "workspace clear");
    }
    if (p->mode == MQH_OP_MATFREE_FP32) {
        block_shapes(p, w);
        const int S = p->fixed_shapes ? (w.S_rows > w.S_cols ? w.S_rows : w.S_cols) : kMaxSlices;
        if ((rc = dalloc(&w.Vg, (size_t)n * kBlkRhs)) || (rc = dalloc(&w.Vh, (size_t)((n + 3) / 4) * kBlkRhs)) ||
            (rc = dalloc(&w.vsc_unit, (size_t)kBlkRhs)) || (rc = dalloc(&w.vsc_data, (size_t)kBlkRhs)) ||
            (rc = dalloc(&w.PB, (size_t)S * kBlkRhs * (size_t)ldn))) {
            multi_free(w);
            return rc;
        }
        launch_fill_f32(w.vsc_unit, kBlkRhs, 16384.0f, s);
        launch_fill_f32(w.vsc_data, kBlkRhs, 1.0f, s);
        LAUNCHCHK("block-product scales");
        if (!p->fixed_shapes) {
            if ((rc = tune_block_shapes(p, w, zc))) {
                multi_free(w);
                return rc;
            }
            // keep only the partials the chosen shapes use (the tuning
            // launches have completed: its last event was waited for)
            const int Sm = w.S_rows > w.S_cols ? w.S_rows : w.S_cols;
            if (Sm < kMaxSlices) {
                dfree(w.PB);
                if ((rc = dalloc(&w.PB, (size_t)Sm * kBlkRhs * (size_t)ldn))) {
                    multi_free(w);
                    return rc;
                }
            }
        }
    }
    w.nz_cap = zc;
    w.ell_cap = lc;
    return MQH_OK;
}

// Y_k = op(A) X_k - shift_k Zs_k for runs k < nz (run k's vectors at
// base + k * stride; shift_k = shift[k * sstr]; no shift term when Zs is
// null).  Stopped runs are skipped.  staged: w.Vg already holds X in the
// sorted FP32 layout (written by the normalisation that produced X).
int block_product(mqh_problem* p, int nz, int trans, const double* X, int64_t xstr, const double* shift,
                  int64_t sstr, const double* Zs, int64_t zstr, double* Y, const GkbState* st, bool timed,
                  bool staged = false, bool unit = true) {
    MultiWs& w = p->mw;
    hipStream_t s = p->stream;
    if (p->mode != MQH_OP_MATFREE_FP32 || nz < 2) {
        for (int k = 0; k < nz; ++k) {
            int rc = op_product(p, trans, X + k * xstr, shift + k * sstr, 0.0, Zs ? Zs + k * zstr : nullptr,
                                Y + k * p->ldn, st ? st + k : nullptr, timed);
            if (rc) return rc;
        }
        return MQH_OK;
    }
    if (!staged) {
        launch_gather_block(X, xstr, nz, p->perm, p->n, st, w.Vg, s);
        LAUNCHCHK("block gather");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            p->pev.push_back(ev);
        }
        e0 = p->pev[p->pev.size() - 2];
        e1 = p->pev[p->pev.size() - 1];
        HIPCHK(hipEventRecord(e0, s));
    }
    const int S = trans ? w.S_cols : w.S_rows;
    const float* vsc = w.vsc_unit;
    if (!unit) {
        launch_block_vscale(w.Vg, p->n, w.vsc_data, s);
        vsc = w.vsc_data;
    }
    launch_split_block(w.Vg, p->n, vsc, w.Vh, s);
    launch_mfh_block(trans, trans ? w.ft_cols : w.ft_rows, p->XS, p->frames, w.Vh, vsc, p->n, p->n_int, S,
                     trans ? w.slice_cols : w.slice_rows, block_entry(op_ec(p), p->blk_tmax), w.PB, p->ldn, s);
    LAUNCHCHK("block product");
    if (timed) HIPCHK(hipEventRecord(e1, s));
    launch_reduce_block(w.PB, p->ldn, S, p->n, nz, p->perm, shift, sstr, Zs, zstr, Y, p->ldn, st, s);
    LAUNCHCHK("block reduction");
    return MQH_OK;
}

// Runs k < nz start from w.X + k ldn (beta_1 w_1 = f).
int run_gkb_multi(mqh_problem* p, int nz, int32_t ell, int32_t reorth, bool timed) {
    MultiWs& w = p->mw;
    hipStream_t s = p->stream;
    const int64_t n = p->n, ldn = p->ldn;
    const int nbq = sumsq_blocks(n);
    const int nbu = update_blocks(n);
    launch_init_state_b(w.st, ell, w.alpha, w.beta, nz, Bz{w.vstr, w.vstr}, s);
    LAUNCHCHK("init state");
    // block products read their operand from w.Vg, which the normalisation
    // writes (columns past nz stay zero)
    const bool blk = p->mode == MQH_OP_MATFREE_FP32 && nz >= 2;
    const int32_t* ip = blk ? p->iperm : nullptr;
    float* vg = blk ? w.Vg : nullptr;
    if (blk) launch_fill_f32(w.Vg, n * kBlkRhs, 0.f, s);
    launch_sumsq_partial_b(w.X, n, w.npart, nbq, w.st, nz, Bz{ldn, w.nstr}, s);
    launch_finalize_scale_b(w.npart, nbq, 0, 0, n, w.alpha, w.beta, w.st, w.X, w.W, ip, vg, nz,
                            Bz{w.nstr, w.vstr, ldn, w.bstr}, s);
    LAUNCHCHK("initial normalisation");
    auto orthonormalize = [&](const double* V, int32_t m, int kind, int32_t j, double* dst) -> int {
        int nparts;
        if (reorth && m > 0) {
            const Bz ub{w.bstr, w.vstr, ldn, w.nstr};
            launch_gemvt_b(V, ldn, n, m, w.Y, w.gpart, w.cvec, w.st, nz, w.bstr, ldn, w.gstr, w.vstr, s);
            if (m <= kFusedCgsMaxCols) {
                launch_update_gemvt_b(V, ldn, n, m, w.cvec, w.Y, w.gpart, w.st, nz, w.bstr, w.vstr, ldn, w.gstr, s);
            } else {
                launch_update_b(V, ldn, n, m, w.cvec, w.Y, nullptr, w.st, nz, ub, s);
                launch_gemvt_b(V, ldn, n, m, w.Y, w.gpart, w.cvec, w.st, nz, w.bstr, ldn, w.gstr, w.vstr, s);
            }
            launch_update_b(V, ldn, n, m, w.cvec, w.Y, w.npart, w.st, nz, ub, s);
            nparts = nbu;
        } else {
            launch_sumsq_partial_b(w.Y, n, w.npart, nbq, w.st, nz, Bz{ldn, w.nstr}, s);
            nparts = nbq;
        }
        launch_finalize_scale_b(w.npart, nparts, kind, j, n, w.alpha, w.beta, w.st, w.Y, dst, ip, vg, nz,
                                Bz{w.nstr, w.vstr, ldn, w.bstr}, s);
        LAUNCHCHK("reorthogonalisation / normalisation");
        return MQH_OK;
    };
    int rc;
    for (int32_t j = 0; j < ell; ++j) {
        double* Wj = w.W + (int64_t)j * ldn;
        double* Zj = w.Z + (int64_t)j * ldn;
        // r = A^T w_j - beta_j z_{j-1}
        if ((rc = block_product(p, nz, 1, Wj, w.bstr, w.beta + j, w.vstr,
                                j > 0 ? w.Z + (int64_t)(j - 1) * ldn : nullptr, w.bstr, w.Y, w.st, timed, blk)))
            return rc;
        if ((rc = orthonormalize(w.Z, j, 1, j, Zj))) return rc;
        // p = A z_j - alpha_j w_j
        if ((rc = block_product(p, nz, 0, Zj, w.bstr, w.alpha + j, w.vstr, Wj, w.bstr, w.Y, w.st, timed, blk)))
            return rc;
        if ((rc = orthonormalize(w.W, j + 1, 2, j, w.W + (int64_t)(j + 1) * ldn))) return rc;
    }
    return MQH_OK;
}

// The Golub-Kahan loop of a group (run_gkb_multi) as a graph: captured on
// the problem's stream at the first call with this group size, ell, reorth
// and row scaling (the captured launches hold the entry constants), replayed
// after that.  The captured launches hold workspace
// addresses, so a workspace reallocation drops the graph (multi_free).
int run_gkb_multi_graph(mqh_problem* p, int nz, int32_t ell, int32_t reorth) {
    MultiWs& w = p->mw;
    hipStream_t s = p->stream;
    if (w.graph != nullptr && (w.g_nz != nz || w.g_ell != ell || w.g_reorth != reorth || w.g_rs != p->rs)) {
        HIPCHK(hipGraphExecDestroy(w.graph));
        w.graph = nullptr;
    }
    if (w.graph == nullptr) {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int rc = run_gkb_multi(p, nz, ell, reorth, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        if (rc != MQH_OK) {
            if (g != nullptr) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        const hipError_t ei = hipGraphInstantiate(&w.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            w.graph = nullptr;
            return hip_fail(ei, "graph instantiation");
        }
        w.g_nz = nz;
        w.g_ell = ell;
        w.g_reorth = reorth;
        w.g_rs = p->rs;
    }
    HIPCHK(hipGraphLaunch(w.graph, s));
    return MQH_OK;
}

// Stage right-hand sides k0 .. k0 + nz - 1 (columns of F, leading dimension
// ldf) into w.X.
int stage_multi(mqh_problem* p, const double* F, int64_t ldf, int k0, int nz, uint32_t flags) {
    MultiWs& w = p->mw;
    const int64_t n = p->n;
    if (!(flags & MQH_FLAG_DEVICE_PTRS))
        for (int k = 0; k < nz; ++k)
            if (!all_finite(F + (int64_t)(k0 + k) * ldf, n)) return fail(MQH_EINVAL, "non-finite right-hand side");
    HIPCHK(copy_strided(w.X, (size_t)p->ldn * sizeof(double), F + (int64_t)k0 * ldf, (size_t)ldf * sizeof(double),
                            (size_t)n * sizeof(double), (size_t)nz, kind_in(flags), p->stream));
    return MQH_OK;
}

// ---------------------------------------------------------------------------
// Full SVD (one-sided block Jacobi on the rows of [A | f]) and the classical
// regularised solutions on it (Algorithm 3; eq. (14)).  Reference path for
// n <= MQH_FULL_MAX_N: every call assembles A in FP64 into its own work
// matrix (n x (n + 1), rows padded to whole 32-row blocks) and frees it.
// ---------------------------------------------------------------------------

struct FullRun {
    int64_t n = 0, ldg = 0, nrow = 0;
    int nblk = 0, npairs = 0, rounds = 0, S = 1;
    int64_t chunk = 0;
    double* G = nullptr;
    int2* pairs = nullptr;
    double* Pg = nullptr;
    double* Pout = nullptr;
    int32_t* flag = nullptr;
    double* off = nullptr;
    double* maxoff = nullptr;
    double* sig = nullptr;
    double* fh = nullptr;
    int32_t* rank = nullptr;
    double* sv = nullptr;
    double* fs = nullptr;
    int32_t* order = nullptr;
    double* tail = nullptr;
    ParamOut* po = nullptr;
    double* f = nullptr;
    int32_t* rowidx = nullptr;  // the sweep's row order (blocks = runs of 32)
    double* rnorm = nullptr;    // row norms of all nrow rows
    double* rtmp = nullptr;
    // conjugate-gradient iterates y, residuals, directions, B q, dot-product terms, x = G^T y (nz data
    // columns each), G^T q partials, scalars, ||f||^2 per data column
    double* cy = nullptr;
    double* cr = nullptr;
    double* cq = nullptr;
    double* cw = nullptr;
    double* ct = nullptr;
    double* cx = nullptr;
    double* cpart = nullptr;
    double* cpc = nullptr;
    double* fn2 = nullptr;
    int inner = 1;  // cyclic Jacobi sweeps per pair and round (at most): kFullMaxInner, or 2 when small
    int cz = 0;     // data columns the solution buffers were allocated for
    size_t cv = 0;  // and their length in doubles (columns times spacing)
    int32_t* pair_ok = nullptr;    // per schedule slot: round at which the pair was last found orthogonal, or -1
    int32_t* blk_stamp = nullptr;  // per block: round of its last rotation, or -1
    int sweeps = 0;
    double final_off = 0.0;
    ~FullRun() {
        dfree(rowidx);
        dfree(rnorm);
        dfree(rtmp);
        dfree(cy);
        dfree(cr);
        dfree(cq);
        dfree(cw);
        dfree(ct);
        dfree(cx);
        dfree(cpart);
        dfree(cpc);
        dfree(fn2);
        dfree(pair_ok);
        dfree(blk_stamp);
        dfree(G);
        dfree(pairs);
        dfree(Pg);
        dfree(Pout);
        dfree(flag);
        dfree(off);
        dfree(maxoff);
        dfree(sig);
        dfree(fh);
        dfree(rank);
        dfree(sv);
        dfree(fs);
        dfree(order);
        dfree(tail);
        dfree(po);
        dfree(f);
    }
};

constexpr int kFullMaxSweeps = 100;
// One cyclic sweep of the 64 x 64 eigensolver per pair and round: rotations
// from a pair's partly diagonalised Gram matrix still orthogonalise its rows
// better each round, later rounds disturb an exact diagonalisation anyway,
// and the outer sweeps barely grow (33 -> 36 at n = 5 000) while a round's
// eigensolver time falls several-fold.
constexpr int kFullMaxInner = 1;
// Small matrices (at most kFullSmallBlocks blocks of 32 rows, as the
// projected problems of the block Golub-Kahan path) take two: there the
// eigensolver is the whole cost of a round, and two sweeps per pair halve the
// outer sweeps (measured on 16-source projected problems: 4 blocks 17 -> 7
// sweeps, 9.7 -> 6.1 ms; 10 blocks 19 -> 11, 28.9 -> 27.9 ms; 14 blocks
// 18 -> 13 but 40 -> 48 ms).
constexpr int kFullSmallBlocks = 10;
// Orthogonality levels of the Jacobi sweeps (relative to ||A||_F): the target
// full_tol(n), and full_floor(n) = twice that.  The measure, computed from
// FP64 Gram entries over n columns, stalls at 16 .. 20 sqrt(n) eps (measured
// at n = 5 000 and 20 000), so the sweeps also end once it is below the floor
// and has not fallen by a quarter in kFullStall sweeps: converged to rounding.
inline double full_tol(int64_t n) { return 16.0 * sqrt((double)n) * DBL_EPSILON; }
inline double full_floor(int64_t n) { return 2.0 * full_tol(n); }
constexpr int kFullStall = 3;
// Fraction of rotated pairs below which a sweep keeps the row order of the
// one before (de Rijk's ordering matters while many pairs rotate).
constexpr double kFullFreeze = 0.05;

constexpr int kFullCgMax = MQH_FULL_CG_MAX;  // conjugate-gradient iterations of the solutions' dual system
constexpr double kFullCgTol = 1e-15;  // stop when sqrt(r^T D^-1 r) falls below this fraction of its start

// Sizes and buffers of a full SVD of an n x n matrix with nrhs data
// columns: G = [M | F] row-major, ldg = n + nrhs rounded up to 64, rows
// padded with zero rows to an even number of 32-row blocks; the block pairs
// of a round-robin tournament.  G is cleared.
// The per-call state of a prepared run: a zero work matrix, no slot found
// orthogonal, no block rotated (so a run can be reused for another matrix of
// the same size).
int full_reset(hipStream_t s, FullRun& r) {
    HIPCHK(hipMemsetAsync(r.G, 0, (size_t)(r.nrow * r.ldg) * sizeof(double), s));
    HIPCHK(hipMemsetAsync(r.pair_ok, 0xff, (size_t)r.rounds * r.npairs * sizeof(int32_t), s));  // -1
    HIPCHK(hipMemsetAsync(r.blk_stamp, 0xff, (size_t)r.nblk * sizeof(int32_t), s));
    r.sweeps = 0;
    r.final_off = 0.0;
    return MQH_OK;
}

int full_prepare(hipStream_t s, FullRun& r, int64_t n, int nrhs) {
    r.n = n;
    r.ldg = round_up(n + nrhs, 64);
    r.nblk = (int)((n + kFsBlock - 1) / kFsBlock);
    if (r.nblk % 2) ++r.nblk;
    r.nrow = (int64_t)r.nblk * kFsBlock;
    r.npairs = r.nblk / 2;
    r.rounds = r.nblk - 1;
    r.inner = r.nblk <= kFullSmallBlocks ? 2 : kFullMaxInner;
    {
        int64_t S = (2048 + r.npairs - 1) / r.npairs;
        const int64_t smax = (n + 63) / 64;
        if (S > smax) S = smax;
        if (S < 1) S = 1;
        r.chunk = round_up((n + S - 1) / S, 64);
        r.S = (int)((n + r.chunk - 1) / r.chunk);
    }
    int rc;
    if ((rc = dalloc(&r.G, (size_t)(r.nrow * r.ldg))) || (rc = dalloc(&r.pairs, (size_t)r.rounds * r.npairs)) ||
        (rc = dalloc(&r.Pg, (size_t)r.npairs * r.S * 4096)) || (rc = dalloc(&r.Pout, (size_t)r.npairs * 4096)) ||
        (rc = dalloc(&r.flag, (size_t)r.npairs)) || (rc = dalloc(&r.off, (size_t)r.rounds * r.npairs)) ||
        (rc = dalloc(&r.maxoff, 2)) || (rc = dalloc(&r.sig, (size_t)n)) || (rc = dalloc(&r.fh, (size_t)n)) ||
        (rc = dalloc(&r.pair_ok, (size_t)r.rounds * r.npairs)) || (rc = dalloc(&r.blk_stamp, (size_t)r.nblk)) ||
        (rc = dalloc(&r.rank, (size_t)n)) || (rc = dalloc(&r.sv, (size_t)n)) || (rc = dalloc(&r.fs, (size_t)n)) ||
        (rc = dalloc(&r.order, (size_t)n)) || (rc = dalloc(&r.tail, (size_t)n + 1)) || (rc = dalloc(&r.po, 1)) ||
        (rc = dalloc(&r.rowidx, (size_t)r.nrow)) ||
        (rc = dalloc(&r.rnorm, (size_t)r.nrow)) || (rc = dalloc(&r.rtmp, (size_t)r.nrow)))
        return rc;
    // round-robin tournament of the blocks: block 0 stays, the others rotate
    std::vector<int2> pr((size_t)r.rounds * r.npairs);
    std::vector<int> pos((size_t)r.nblk);
    for (int k = 0; k < r.nblk; ++k) pos[(size_t)k] = k;
    for (int rd = 0; rd < r.rounds; ++rd) {
        for (int k = 0; k < r.npairs; ++k) {
            const int a = pos[(size_t)k], b = pos[(size_t)(r.nblk - 1 - k)];
            pr[(size_t)rd * r.npairs + k] = make_int2(a, b);
        }
        const int last = pos[(size_t)(r.nblk - 1)];
        for (int k = r.nblk - 1; k > 1; --k) pos[(size_t)k] = pos[(size_t)(k - 1)];
        pos[1] = last;
    }
    HIPCHK(hipMemcpyAsync(r.pairs, pr.data(), pr.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    int rc2;
    if ((rc2 = full_reset(s, r))) return rc2;
    HIPCHK(hipStreamSynchronize(s));  // pr is a local
    return MQH_OK;
}

// Jacobi sweeps on the filled G (n matrix columns, nrhs data columns), each
// on the rows ordered by decreasing norm (kept from the sweep before once
// fewer than kFullFreeze of the pairs rotate; a pair whose rows have not
// changed since it was last found orthogonal is then left out), until in a
// whole sweep every pair of rows has the component of the smaller along
// the larger at most full_tol(n) ||M||_F, or stalls below full_floor(n)
// ||M||_F (or kFullMaxSweeps); then sigma and the first data column f^
// (input row order) and their descending order.
int full_sweeps(hipStream_t s, FullRun& r, int64_t n, int nrhs) {
    const double tol = full_tol(n);
    const int64_t slots = (int64_t)r.rounds * r.npairs;
    std::vector<double> rn((size_t)r.nrow);
    std::vector<int32_t> idx((size_t)r.nrow), prev;
    double inv_f = 0.0;
    r.sweeps = 0;
    // MQH_TRACE_FULL=1 prints one line per sweep to stderr (diagnostics only)
    const char* tr = getenv("MQH_TRACE_FULL");
    const bool trace = tr != nullptr && tr[0] == '1';
    auto t0 = std::chrono::steady_clock::now();
    const double floor_off = full_floor(n);
    double best = HUGE_VAL;
    int stall = 0;
    bool frozen = false;  // row order fixed (few pairs still rotate)
    for (int sw = 0; sw < kFullMaxSweeps; ++sw) {
        int same = 1;
        if (!frozen) {
            // de Rijk's ordering: rows by decreasing norm (stable), blocks of 32
            launch_fs_norms(r.G, r.ldg, r.nrow, n, r.rnorm, r.rtmp, s);
            LAUNCHCHK("full SVD: row norms");
            HIPCHK(hipMemcpyAsync(rn.data(), r.rnorm, (size_t)r.nrow * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (sw == 0) {
                // ||M||_F (invariant under the rotations)
                double fro2 = 0.0;
                for (double v : rn) fro2 += v * v;
                if (!(fro2 > 0.0) || !isfinite(fro2)) return fail(MQH_EDEVICE, "full SVD: zero or non-finite matrix");
                inv_f = 1.0 / sqrt(fro2);
            }
            for (int64_t i = 0; i < r.nrow; ++i) idx[(size_t)i] = (int32_t)i;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t a, int32_t b) { return rn[(size_t)a] > rn[(size_t)b]; });
            same = idx == prev ? 1 : 0;
            if (!same) {
                prev = idx;
                HIPCHK(hipMemcpyAsync(r.rowidx, prev.data(), prev.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                      s));
            }
        }
        for (int rd = 0; rd < r.rounds; ++rd) {
            const int2* prd = r.pairs + (int64_t)rd * r.npairs;
            const int64_t slot0 = (int64_t)rd * r.npairs;
            const int32_t g = sw * r.rounds + rd;
            launch_fs_gram(r.G, r.ldg, n, r.rowidx, prd, r.npairs, r.S, r.chunk, r.Pg, r.pair_ok, r.blk_stamp, slot0,
                           same, s);
            launch_fs_eig(r.Pg, r.S, r.npairs, tol, inv_f, r.inner, r.Pout, r.flag, r.off + slot0, prd,
                          r.pair_ok, r.blk_stamp, slot0, g, same, s);
            launch_fs_update(r.G, r.ldg, n + nrhs, r.rowidx, prd, r.npairs, r.Pout, r.flag, s);
        }
        LAUNCHCHK("full SVD: Jacobi sweep");
        launch_fs_maxoff(r.off, slots, tol, r.maxoff, s);
        double mo[2] = {0.0, 0.0};
        HIPCHK(hipMemcpyAsync(mo, r.maxoff, sizeof(mo), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        r.sweeps = sw + 1;
        r.final_off = mo[0];
        if (trace) {
            const auto t1 = std::chrono::steady_clock::now();
            fprintf(stderr, "[mqh full] sweep %d off %.3e rotated %.0f of %lld pairs%s %.1f ms\n", sw + 1, mo[0], mo[1],
                    (long long)slots, same ? " (order kept)" : "",
                    std::chrono::duration<double, std::milli>(t1 - t0).count());
            t0 = t1;
        }
        if (!(mo[0] > tol)) break;
        // once fewer than 5% of the pairs still rotate, keep the row order: blocks stay the same,
        // and pairs whose rows have not changed are left out
        if (mo[1] < kFullFreeze * (double)slots) frozen = true;
        if (mo[0] < 0.75 * best) {
            best = mo[0];
            stall = 0;
        } else if (++stall >= kFullStall && !(mo[0] > floor_off)) {
            break;
        }
    }
    launch_fs_norms(r.G, r.ldg, n, n, r.sig, r.fh, s);
    launch_fs_rank(r.sig, r.fh, n, r.rank, r.sv, r.fs, r.order, s);
    LAUNCHCHK("full SVD: singular values");
    return MQH_OK;
}

// Assembles [A | f] (f already staged in r.f, or zero) and runs the sweeps.
int full_svd_run(mqh_problem* p, FullRun& r) {
    hipStream_t s = p->stream;
    const int64_t n = p->n;
    int rc;
    if ((rc = full_prepare(s, r, n, 1))) return rc;
    launch_assemble(p->X64, n, p->n_int, r.ldg, p->ec, r.G, s);
    LAUNCHCHK("full SVD: assembly");
    launch_fs_setf(r.G, r.ldg, n, r.f, s);
    LAUNCHCHK("full SVD: data column");
    HIPCHK(hipEventRecord(p->ev[1], s));
    if ((rc = full_sweeps(s, r, n, 1))) return rc;
    HIPCHK(hipEventRecord(p->ev[2], s));
    HIPCHK(hipEventRecord(p->ev[3], s));
    return MQH_OK;
}

// The solutions x = G^T y of the Tikhonov (method 1) or TSVD (method 0) dual
// systems by preconditioned conjugate gradients (the kernels' comment gives
// the system) for nz data columns at once: column z's data fh + z vs
// (physical row order) and choice po + z; rows of rank >= rcap are left
// out.  Every column runs until all have reached the tolerance (or the
// cap); a column past its own tolerance keeps taking steps whose size has
// fallen with its residual.  x_z in r.cx + z vs; then po[z].rho =
// ||M x_z - f_z|| and po[z].eta = ||x_z||.  iters[z]: the iteration at which
// column z reached its tolerance (or the cap, converged[z] false).
int full_solution(hipStream_t s, FullRun& r, int64_t n, int32_t method, const double* fh, int64_t vs, ParamOut* po,
                  int64_t rcap, int nz, int* iters, bool* converged) {
    int rc;
    const int chunks = fs_gemvt_chunks(n);
    if (vs < n) return fail(MQH_EINVAL, "full problem: solution columns closer than n apart");
    const size_t v = (size_t)vs * (size_t)nz;
    if (r.cq != nullptr && (r.cz < nz || r.cv < v))
        return fail(MQH_EINVAL, "full problem: more solution columns than allocated");
    if (r.cq == nullptr) {
        if ((rc = dalloc(&r.cy, v)) || (rc = dalloc(&r.cr, v)) || (rc = dalloc(&r.cq, v)) || (rc = dalloc(&r.cw, v)) ||
            (rc = dalloc(&r.ct, v)) || (rc = dalloc(&r.cx, v)) ||
            (rc = dalloc(&r.cpart, (size_t)nz * (size_t)chunks * (size_t)n)) || (rc = dalloc(&r.cpc, 4 * (size_t)nz)))
            return rc;
        r.cz = nz;
        r.cv = v;
    }
    launch_fs_pcg_start(r.sig, fh, r.rank, n, method, rcap, po, vs, r.cy, r.cr, r.cq, r.ct, r.cpc, 2, nz, s);
    LAUNCHCHK("full problem: solution start");
    std::vector<double> pc((size_t)4 * nz), stop((size_t)nz);
    HIPCHK(hipMemcpyAsync(pc.data(), r.cpc, pc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int open = 0;
    for (int z = 0; z < nz; ++z) {
        const double rz0 = pc[(size_t)4 * z + 2];
        if (!isfinite(rz0)) return fail(MQH_EDEVICE, "full problem: non-finite right-hand side of the solution");
        stop[(size_t)z] = kFullCgTol * kFullCgTol * rz0;
        iters[z] = 0;
        converged[z] = !(rz0 > 0.0);
        open += converged[z] ? 0 : 1;
    }
    const char* tr = getenv("MQH_TRACE_FULL");
    const bool trace = tr != nullptr && tr[0] == '1';
    int it = 0;
    while (open > 0 && it < kFullCgMax) {
        const int cur = 2 + (it & 1), nxt = 2 + ((it + 1) & 1);
        launch_fs_pcg_iter(r.G, r.ldg, n, r.sig, r.rank, method, rcap, po, vs, r.cpc, cur, nxt, r.cy, r.cr, r.cq,
                           r.cw, r.ct, r.cpart, r.cx, nz, s);
        LAUNCHCHK("full problem: solution iteration");
        HIPCHK(hipMemcpyAsync(pc.data(), r.cpc, pc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ++it;
        for (int z = 0; z < nz; ++z) {
            const double rz = pc[(size_t)4 * z + nxt];
            if (!isfinite(rz)) return fail(MQH_EDEVICE, "full problem: non-finite solution iterate");
            if (!converged[z] && !(rz > stop[(size_t)z])) {
                converged[z] = true;
                iters[z] = it;
                --open;
            }
        }
        if (trace && (it % 8 == 0 || it < 8))
            fprintf(stderr, "[mqh full] cg %d: %d of %d columns still open\n", it, open, nz);
        if (open == 0) break;
        launch_fs_pcg_dir(r.sig, r.rank, n, method, rcap, po, vs, r.cpc, cur, nxt, r.cr, r.cq, nz, s);
    }
    for (int z = 0; z < nz; ++z)
        if (!converged[z]) iters[z] = it;
    launch_fs_gemvt(r.G, r.ldg, n, r.cy, vs, r.cpart, r.cx, nz, s);
    launch_fs_solution_norms(r.G, r.ldg, n, r.cx, fh, vs, r.ct, r.cw, r.cpc, po, nz, s);
    LAUNCHCHK("full problem: solution");
    return MQH_OK;
}

int stage_in(double* dst, const double* src, int64_t count, uint32_t flags, hipStream_t s) {
    if (count <= 0) return MQH_OK;
    if (!(flags & MQH_FLAG_DEVICE_PTRS) && !all_finite(src, count)) return fail(MQH_EINVAL, "non-finite input");
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)count * sizeof(double), kind_in(flags), s));
    return MQH_OK;
}

int check_problem(const mqh_problem* p) {
    if (p == nullptr) return fail(MQH_EINVAL, "NULL problem");
    return MQH_OK;
}

int check_opts(const mqh_problem* p, const mqh_solve_opts* opts) {
    const int32_t ell = opts->ell;
    if (ell < 1 || ell > p->n || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= min(n, MQH_MAX_ELL)");
    if (opts->reorth != 0 && opts->reorth != 1) return fail(MQH_EINVAL, "reorth must be 0 or 1");
    if (opts->method != MQH_METHOD_INE_TSVD && opts->method != MQH_METHOD_HKT && opts->method != MQH_METHOD_LSQR)
        return fail(MQH_EINVAL, "method");
    if (opts->rule < MQH_RULE_GCV || opts->rule > MQH_RULE_WGCV) return fail(MQH_EINVAL, "rule");
    if (opts->row_scale != 0 && opts->row_scale != 1) return fail(MQH_EINVAL, "row_scale must be 0 or 1");
    if (opts->method == MQH_METHOD_LSQR && opts->rule == MQH_RULE_WGCV)
        return fail(MQH_EINVAL, "the weighted GCV rule applies to HKT and Ine-TSVD");
    if (opts->rule == MQH_RULE_WGCV && !(opts->gcv_weight > 0.0 && opts->gcv_weight <= 1.0))
        return fail(MQH_EINVAL, "gcv_weight must be in (0, 1]");
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    if (J < 3 || J > kMaxGrid) return fail(MQH_EINVAL, "n_grid must be 0 or in [3, 4096]");
    if (opts->method == MQH_METHOD_HKT && opts->rule == MQH_RULE_FIXED &&
        (!isfinite(opts->lambda_fixed) || opts->lambda_fixed < 0.0))
        return fail(MQH_EINVAL, "lambda_fixed must be finite and >= 0");
    if (opts->method != MQH_METHOD_HKT && opts->rule == MQH_RULE_FIXED && (opts->k_trunc < 1 || opts->k_trunc > ell))
        return fail(MQH_EINVAL, "k_trunc must be in [1, ell]");
    return MQH_OK;
}

void clear_info(mqh_solve_info* info) {
    if (info) memset(info, 0, sizeof(*info));
}

// ---------------------------------------------------------------------------
// Block Golub-Kahan for s <= 16 right-hand sides sharing one Krylov space
// (Algorithm 1 with an n x s starting block) and the block Tikhonov
// solutions on it.  Bases W (n x (ell + 1) s) and Z (n x ell s) are
// column-major with leading dimension ldn, block j at column j s.
// ---------------------------------------------------------------------------

struct BlockWs {
    double* W = nullptr;
    double* Z = nullptr;
    double* P = nullptr;     // ldn x 16 work block
    double* part = nullptr;  // split-K partials of V^T P
    double* c = nullptr;     // m x 16 coefficients
    double* G = nullptr;     // 16 x 16 Gram matrix
    double* Rinv = nullptr;  // 16 x 16
    double* Racc = nullptr;  // 16 x 16 accumulated R
    double* mat = nullptr;   // two 16 x 16 shift blocks (c layout), written by the QR checks
    int32_t* status = nullptr;
    double* Cd = nullptr;    // C ((ell + 1) s x ell s, row-major) on the device
    double* E1d = nullptr;   // E_1 (s x s)
    BlkState* bs = nullptr;  // breakdown state of the run
    ~BlockWs() {
        dfree(Cd);
        dfree(E1d);
        dfree(bs);
        dfree(W);
        dfree(Z);
        dfree(P);
        dfree(part);
        dfree(c);
        dfree(G);
        dfree(Rinv);
        dfree(Racc);
        dfree(mat);
        dfree(status);
    }
};

int block_alloc(mqh_problem* p, BlockWs& b, int32_t s, int32_t ell) {
    const int64_t ldn = p->ldn;
    const int32_t mmax = (ell + 1) * s;
    int64_t chunk;
    int64_t most = 0;  // largest chunks x m over the m the process uses
    for (int32_t m = s; m <= mmax; m += s) {
        const int64_t q = (int64_t)blk_chunks(p->n, m, &chunk) * m;
        if (q > most) most = q;
    }
    int rc;
    if ((rc = dalloc(&b.W, (size_t)((int64_t)mmax * ldn))) || (rc = dalloc(&b.Z, (size_t)((int64_t)ell * s * ldn))) ||
        (rc = dalloc(&b.P, (size_t)(kBlkRhs * ldn))) || (rc = dalloc(&b.part, (size_t)(most * kBlkRhs))) ||
        (rc = dalloc(&b.c, (size_t)mmax * kBlkRhs)) || (rc = dalloc(&b.G, kBlkRhs * kBlkRhs)) ||
        (rc = dalloc(&b.Rinv, kBlkRhs * kBlkRhs)) || (rc = dalloc(&b.Racc, kBlkRhs * kBlkRhs)) ||
        (rc = dalloc(&b.mat, 2 * kBlkRhs * kBlkRhs)) || (rc = dalloc(&b.status, 1)) ||
        (rc = dalloc(&b.Cd, (size_t)mmax * (size_t)ell * s)) || (rc = dalloc(&b.E1d, kBlkRhs * kBlkRhs)) ||
        (rc = dalloc(&b.bs, 1)))
        return rc;
    hipStream_t st = p->stream;
    HIPCHK(hipMemsetAsync(b.W, 0, (size_t)mmax * ldn * sizeof(double), st));
    HIPCHK(hipMemsetAsync(b.Z, 0, (size_t)ell * s * ldn * sizeof(double), st));
    HIPCHK(hipMemsetAsync(b.P, 0, (size_t)kBlkRhs * ldn * sizeof(double), st));
    return MQH_OK;
}

// Workspaces of the block calls, kept on the problem between calls: at the
// sizes of the block solves the allocations and frees of a call (about 50,
// each free waiting for the device) cost more than a tenth of the call.  The
// block bases for (s, ell) with the projected solutions Y (ell s x 16) and
// singular values, and the projected problem's run for its size (m, s) with
// its per-source buffers.
// Buffers of the band path of a projected problem of N = ell s columns and s
// sources (band_kernels.hip): the chase's reflectors and step offsets, the
// bidiagonal, the SVD workspace, values and vectors, the data G, H = U g,
// U^T H, F~ (column-major per source), yhat, ||b_k||^2, the parameter
// choices and the acceptance status.
struct BandRun {
    int N = 0, s = 0, T = 0, ntask = 0;
    double *RR = nullptr, *LL = nullptr, *d = nullptr, *e = nullptr, *ws = nullptr, *sv = nullptr, *V = nullptr,
           *ftil = nullptr, *G = nullptr, *H = nullptr, *Wt = nullptr, *F = nullptr, *Yh = nullptr, *fn2 = nullptr,
           *tail = nullptr;
    int32_t *toff = nullptr, *status = nullptr;
    ParamOut* po = nullptr;
    ~BandRun() {
        dfree(RR);
        dfree(LL);
        dfree(d);
        dfree(e);
        dfree(ws);
        dfree(sv);
        dfree(V);
        dfree(ftil);
        dfree(G);
        dfree(H);
        dfree(Wt);
        dfree(F);
        dfree(Yh);
        dfree(fn2);
        dfree(tail);
        dfree(toff);
        dfree(status);
        dfree(po);
    }
};

struct BlockCache {
    std::unique_ptr<BlockWs> ws;
    std::unique_ptr<BandRun> br;  // the band path's buffers for its (N, s)
    int32_t s = 0, ell = 0;
    double* Y = nullptr;
    double* sv = nullptr;
    std::unique_ptr<FullRun> fr;
    int64_t m = 0;
    int32_t fs = 0;
    double* fh = nullptr;    // data columns, m x s
    double* fsrt = nullptr;  // the same in descending singular-value order
    double* tail = nullptr;  // (m + 1) x s
    double* fn2 = nullptr;   // ||f_k||^2
    ParamOut* po = nullptr;
    void drop_ws() {
        ws.reset();
        dfree(Y);
        dfree(sv);
        Y = sv = nullptr;
    }
    void drop_run() {
        fr.reset();
        dfree(fh);
        dfree(fsrt);
        dfree(tail);
        dfree(fn2);
        dfree(po);
        fh = fsrt = tail = fn2 = nullptr;
        po = nullptr;
    }
    ~BlockCache() {
        drop_run();
        drop_ws();
    }
};

void block_cache_free(BlockCache* c) { delete c; }

// The block workspace for s sources and ell steps, from the cache or newly
// allocated; bases cleared either way.
int block_ws(mqh_problem* p, int32_t s, int32_t ell, BlockWs** out) {
    if (p->bc == nullptr) p->bc = new BlockCache;
    BlockCache& c = *p->bc;
    int rc;
    if (c.ws && c.s == s && c.ell == ell) {
        const int64_t ldn = p->ldn;
        hipStream_t st = p->stream;
        HIPCHK(hipMemsetAsync(c.ws->W, 0, (size_t)(ell + 1) * s * ldn * sizeof(double), st));
        HIPCHK(hipMemsetAsync(c.ws->Z, 0, (size_t)ell * s * ldn * sizeof(double), st));
        HIPCHK(hipMemsetAsync(c.ws->P, 0, (size_t)kBlkRhs * ldn * sizeof(double), st));
    } else {
        c.drop_ws();
        c.ws.reset(new BlockWs);
        c.s = s;
        c.ell = ell;
        if ((rc = block_alloc(p, *c.ws, s, ell)) || (rc = dalloc(&c.Y, (size_t)ell * s * kBlkRhs)) ||
            (rc = dalloc(&c.sv, (size_t)ell * s))) {
            c.drop_ws();
            c.s = c.ell = 0;
            return rc;
        }
    }
    *out = c.ws.get();
    return MQH_OK;
}

// Q R = X in place (X: n x s, leading dimension ldn) by shifted Cholesky QR
// three times; R (s x s, row-major, upper triangular) to the host.  *bad is
// set when a Cholesky factorisation fails (X numerically zero or not finite).
// Cholesky QR of the s columns of X in place (three passes, the first
// shifted), then the breakdown test and the bookkeeping of the factor on
// the device (k_blk_check: kind 0 for E_1, 1 for D_j, 2 for E_{j+1}); the
// factor's transpose goes to shift slot `slot` of b.mat.
void block_qr(mqh_problem* p, BlockWs& b, double* X, int32_t s, int32_t kind, int32_t j, int32_t ell, int slot) {
    hipStream_t st = p->stream;
    const int64_t n = p->n, ldn = p->ldn;
    launch_blk_eye(b.Racc, b.status, st);
    for (int pass = 0; pass < 3; ++pass) {
        launch_blk_gemvt(X, ldn, n, s, X, ldn, s, b.part, b.G, st);
        launch_blk_chol(b.G, s, n, pass == 0 ? 1 : 0, b.Rinv, b.Racc, b.status, st);
        launch_blk_update(X, ldn, n, s, b.Rinv, kBlkRhs, 1, X, ldn, s, 0, st);
    }
    launch_blk_check(b.Racc, b.status, s, kind, j, (double)n * DBL_EPSILON, b.bs, b.Cd, (int64_t)ell * s, b.E1d,
                     b.mat + slot * kBlkRhs * kBlkRhs, st);
}

// X -= V M with M the device coefficients in shift slot `slot` of b.mat (the
// transpose of the QR factor k_blk_check left there).
void block_shift_dev(mqh_problem* p, BlockWs& b, const double* V, int32_t s, double* X, int slot) {
    launch_blk_update(V, p->ldn, p->n, s, b.mat + slot * kBlkRhs * kBlkRhs, kBlkRhs, 1, X, p->ldn, s, 1, p->stream);
}

// X -= V (V^T X) twice, V the first m columns of a basis.
void block_cgs2(mqh_problem* p, BlockWs& b, const double* V, int32_t m, int32_t s, double* X) {
    if (m <= 0) return;
    hipStream_t st = p->stream;
    for (int pass = 0; pass < 2; ++pass) {
        launch_blk_gemvt(V, p->ldn, p->n, m, X, p->ldn, s, b.part, b.c, st);
        launch_blk_update(V, p->ldn, p->n, m, b.c, kBlkRhs, 1, X, p->ldn, s, 1, st);
    }
}

// The block recurrence from the block already in W's first s columns:
// W_1 E_1 = F; Z_j D_j^T = A^T W_j - Z_{j-1} E_j^T; W_{j+1} E_{j+1} =
// A Z_j - W_j D_j, each right side reorthogonalised against all earlier
// blocks of its basis (CGS2) before its QR.  C (host, (ell + 1) s x ell s
// row-major; left empty when host_c is false, the device copy b.Cd holds it
// either way) receives D_j and E_{j+1}; E1 (s x s) the data's factor.  A QR
// with a diagonal entry of R at most n eps times the largest diagonal entry
// of the D and E blocks so far (E_1 left out) is a breakdown: at a D block
// *ell_done = j - 1 (flag 1), at an E block *ell_done = j with E_{j+1} = 0
// (flag 2).  The tests run on the device and the whole run is enqueued
// without a synchronisation; steps after a breakdown still run but write
// nothing into C, and the basis columns past the kept steps are cleared at
// the end.
int run_gkb_block(mqh_problem* p, BlockWs& b, int32_t s, int32_t ell, std::vector<double>& C, double* E1,
                  int32_t* ell_done, int32_t* flag, bool host_c = true) {
    hipStream_t st = p->stream;
    const int64_t ldn = p->ldn;
    const int64_t ldc = (int64_t)ell * s;
    const size_t csize = (size_t)((ell + 1) * s) * (size_t)ldc;
    C.assign(host_c ? csize : 0, 0.0);
    HIPCHK(hipMemsetAsync(b.Cd, 0, csize * sizeof(double), st));
    HIPCHK(hipMemsetAsync(b.bs, 0, sizeof(BlkState), st));
    block_qr(p, b, b.W, s, 0, 0, ell, 0);
    for (int32_t j = 1; j <= ell; ++j) {
        double* Wj = b.W + (int64_t)(j - 1) * s * ldn;
        double* Zj = b.Z + (int64_t)(j - 1) * s * ldn;
        // P = A^T W_j - Z_{j-1} E_j^T, reorthogonalised against Z_1 .. Z_{j-1}
        int rc;
        if ((rc = block_product(p, s, 1, Wj, ldn, nullptr, 0, nullptr, 0, b.P, nullptr, false))) return rc;
        if (j > 1) block_shift_dev(p, b, Zj - (int64_t)s * ldn, s, b.P, 0);
        block_cgs2(p, b, b.Z, (j - 1) * s, s, b.P);
        block_qr(p, b, b.P, s, 1, j, ell, 1);  // D_j = R^T into C; the shift below reads slot 1
        HIPCHK(hipMemcpyAsync(Zj, b.P, (size_t)s * ldn * sizeof(double), hipMemcpyDeviceToDevice, st));
        // Q = A Z_j - W_j D_j, reorthogonalised against W_1 .. W_j
        if ((rc = block_product(p, s, 0, Zj, ldn, nullptr, 0, nullptr, 0, b.P, nullptr, false))) return rc;
        block_shift_dev(p, b, Wj, s, b.P, 1);
        block_cgs2(p, b, b.W, j * s, s, b.P);
        block_qr(p, b, b.P, s, 2, j, ell, 0);  // E_{j+1} = R, the next step's shift
        HIPCHK(hipMemcpyAsync(Wj + (int64_t)s * ldn, b.P, (size_t)s * ldn * sizeof(double), hipMemcpyDeviceToDevice,
                              st));
    }
    LAUNCHCHK("block Golub-Kahan");
    BlkState h{};
    HIPCHK(hipMemcpyAsync(&h, b.bs, sizeof(BlkState), hipMemcpyDeviceToHost, st));
    if (host_c) HIPCHK(hipMemcpyAsync(C.data(), b.Cd, csize * sizeof(double), hipMemcpyDeviceToHost, st));
    double E1h[kBlkRhs * kBlkRhs];
    HIPCHK(hipMemcpyAsync(E1h, b.E1d, (size_t)s * s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // a zero source fails the Cholesky step; sources dependent to working precision leave E_1 a
    // diagonal entry at the rounding level (or, by rounding, fail it too): either way W_1 would
    // carry a direction of rounding noise, so both are rejected
    if (h.invalid)
        return fail(MQH_EINVAL, "block Golub-Kahan: the right-hand sides are zero or linearly dependent");
    for (int i = 0; i < s * s; ++i) E1[i] = E1h[i];
    *ell_done = h.stopped ? h.ell_done : ell;
    *flag = h.stopped ? h.flag : 0;
    if (h.stopped) {
        // the kept basis: W_1 .. W_{ell_done + 1} after a D breakdown, W_1 .. W_{ell_done} after an E
        // breakdown (E_{ell_done + 1} = 0), Z_1 .. Z_{ell_done}; the rest is cleared
        const int64_t wk = (int64_t)(*ell_done + (*flag == 1 ? 1 : 0)) * s;
        const int64_t zk = (int64_t)(*ell_done) * s;
        HIPCHK(hipMemsetAsync(b.W + wk * ldn, 0, (size_t)(((int64_t)(ell + 1) * s - wk) * ldn) * sizeof(double), st));
        HIPCHK(hipMemsetAsync(b.Z + zk * ldn, 0, (size_t)(((int64_t)ell * s - zk) * ldn) * sizeof(double), st));
    }
    return MQH_OK;
}

// The projected problem by the band path: the chase of C^T (C on the
// device, (ell + 1) s x ell s at leading dimension ldc; E1 on the device,
// s x s row-major), the multisection SVD of the bidiagonal, F~ for the s
// sources, the parameter choices (as block_projected) and the solutions into
// Y.  *ok = false when the SVD failed its acceptance test (Y, sv untouched
// in meaning; the caller takes the Jacobi path).
int band_projected(mqh_problem* p, const double* Cd, int64_t ldc, const double* E1d, int32_t s, int32_t ell,
                   int32_t rule, int32_t J, double lambda_fixed, double* Y, double* sv_out,
                   std::vector<ParamOut>& po_h, bool* ok) {
    hipStream_t st = p->stream;
    const int N = ell * s, Mc = N + s;
    BlockCache& bc = *p->bc;
    int rc;
    if (!bc.br || bc.br->N != N || bc.br->s != s) {
        bc.br.reset(new BandRun);
        BandRun& r = *bc.br;
        r.N = N;
        r.s = s;
        r.ntask = band_ntasks(N, s, &r.T);
        const size_t nt = (size_t)(r.ntask > 0 ? r.ntask : 1) * (size_t)(s + 1);
        if ((rc = dalloc(&r.RR, nt)) || (rc = dalloc(&r.LL, nt)) || (rc = dalloc(&r.d, (size_t)N)) ||
            (rc = dalloc(&r.e, (size_t)N)) || (rc = dalloc(&r.ws, svd_ws_doubles(N))) ||
            (rc = dalloc(&r.sv, (size_t)N)) || (rc = dalloc(&r.V, (size_t)N * N)) ||
            (rc = dalloc(&r.ftil, (size_t)N + 1)) || (rc = dalloc(&r.G, (size_t)N * kBlkRhs)) ||
            (rc = dalloc(&r.H, (size_t)N * kBlkRhs)) || (rc = dalloc(&r.Wt, (size_t)N * kBlkRhs)) ||
            (rc = dalloc(&r.F, (size_t)N * kBlkRhs)) || (rc = dalloc(&r.Yh, (size_t)N * kBlkRhs)) ||
            (rc = dalloc(&r.fn2, (size_t)kBlkRhs)) || (rc = dalloc(&r.tail, (size_t)(Mc + 1) * kBlkRhs)) ||
            (rc = dalloc(&r.toff, (size_t)r.T + 1)) || (rc = dalloc(&r.status, 1)) ||
            (rc = dalloc(&r.po, (size_t)kBlkRhs))) {
            bc.br.reset();
            return rc;
        }
    }
    BandRun& r = *bc.br;
    launch_band_chase(Cd, ldc, N, s, r.T, r.RR, r.LL, r.toff, r.d, r.e, st);
    launch_band_data(E1d, N, s, r.RR, r.toff, r.T, r.d, r.e, r.ws, r.G, r.fn2, st);
    LAUNCHCHK("block projected problem: band reduction");
    launch_msvd_core(N, r.ws, r.sv, r.ftil, r.V, N, r.status, st);
    LAUNCHCHK("block projected problem: SVD");
    const double* U = r.ws;  // the SVD workspace starts with U (rows u_j, ld N)
    launch_band_mm(0, U, N, N, s, r.G, nullptr, nullptr, nullptr, r.H, st);
    launch_band_mm(1, U, N, N, s, r.H, nullptr, nullptr, nullptr, r.Wt, st);
    launch_band_mm(2, U, N, N, s, r.Wt, r.H, nullptr, nullptr, r.F, st);
    launch_full_param(r.sv, r.F, Mc, N, r.fn2, N, 1, rule == MQH_RULE_FIXED ? 2 : 0, J, lambda_fixed, 0, r.tail, r.po,
                      s, st);
    launch_band_mm(3, r.V, N, N, s, r.F, nullptr, r.sv, r.po, r.Yh, st);
    launch_band_solve(r.Yh, N, s, r.LL, r.toff, r.T, Y, st);
    LAUNCHCHK("block projected problem: choices and solutions");
    if (sv_out) HIPCHK(hipMemcpyAsync(sv_out, r.sv, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, st));
    int32_t status = -1;
    po_h.assign((size_t)s, ParamOut{});
    HIPCHK(hipMemcpyAsync(&status, r.status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(po_h.data(), r.po, (size_t)s * sizeof(ParamOut), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *ok = status == 0;
    return MQH_OK;
}

// Block Tikhonov on the projected problem: per source k, min ||C y - b_k||^2
// + lambda_k^2 ||y||^2 with b_k = (E_1 e_k; 0), through the full-SVD path on
// the square (ell + 1) s matrix [C | 0] with the s columns b_k beside it
// (the zero columns add s zero singular values, which the rank cap ell s
// keeps out of the choice and the solution); lambda_k by the full-problem
// GCV on (ell + 1) s rows (rule GCV) or lambda_fixed (rule FIXED).  Y
// (device, ell s x 16, row col = Y + 16 col) receives y_k in column k;
// per-source records in po_h / iters / conv; sv (device, ell s, NULL
// allowed) the singular values.
int block_projected(mqh_problem* p, const double* Cd, int64_t ldcd, const double* E1d, const double* E1, int32_t s,
                    int32_t ell, int32_t rule, int32_t J, double lambda_fixed, double* Y, double* sv,
                    std::vector<ParamOut>& po_h, std::vector<int>& iters, std::vector<char>& conv, int32_t* sweeps) {
    hipStream_t st = p->stream;
    const int64_t m = (int64_t)(ell + 1) * s, ls = (int64_t)ell * s;
    BlockCache& bc = *p->bc;  // made by block_ws
    int rc;
    if (bc.fr && bc.m == m && bc.fs == s) {
        if ((rc = full_reset(st, *bc.fr))) return rc;
    } else {
        bc.drop_run();
        bc.fr.reset(new FullRun);
        bc.m = m;
        bc.fs = s;
        if ((rc = full_prepare(st, *bc.fr, m, s)) || (rc = dalloc(&bc.fh, (size_t)(m * s))) ||
            (rc = dalloc(&bc.fsrt, (size_t)(m * s))) || (rc = dalloc(&bc.tail, (size_t)((m + 1) * s))) ||
            (rc = dalloc(&bc.fn2, (size_t)s)) || (rc = dalloc(&bc.po, (size_t)s))) {
            bc.drop_run();
            bc.m = 0;
            return rc;
        }
    }
    FullRun& r = *bc.fr;
    launch_blk_fill_g(Cd, ldcd, m, ls, E1d, s, r.G, r.ldg, st);
    LAUNCHCHK("block projected problem: work matrix");
    if ((rc = full_sweeps(st, r, m, s))) return rc;
    *sweeps = r.sweeps;
    if (sv) HIPCHK(hipMemcpyAsync(sv, r.sv, (size_t)ls * sizeof(double), hipMemcpyDeviceToDevice, st));
    // the sources' data columns, their sorted order, the choices and the solutions, all at once
    double* fh_all = bc.fh;
    double* fs_all = bc.fsrt;
    double* tail_all = bc.tail;
    double* fn2 = bc.fn2;
    ParamOut* po_all = bc.po;
    std::vector<double> fn2h((size_t)s, 0.0);
    for (int k = 0; k < s; ++k)
        for (int i = 0; i < s; ++i) fn2h[(size_t)k] += E1[i * s + k] * E1[i * s + k];
    HIPCHK(hipMemcpyAsync(fn2, fn2h.data(), (size_t)s * sizeof(double), hipMemcpyHostToDevice, st));
    launch_fs_col(r.G, r.ldg, m, m, m, fh_all, s, st);
    launch_fs_rank(r.sig, fh_all, m, r.rank, r.sv, r.fs, r.order, st);
    launch_fs_gather(r.rank, fh_all, m, m, fs_all, s, st);
    launch_full_param(r.sv, fs_all, m, ls, fn2, m, 1, rule == MQH_RULE_FIXED ? 2 : 0, J, lambda_fixed, 0, tail_all,
                      po_all, s, st);
    LAUNCHCHK("block projected problem: parameter choice");
    iters.assign((size_t)s, 0);
    std::vector<int> it((size_t)s, 0);
    bool cv[kBlkRhs];
    if ((rc = full_solution(st, r, m, 1, fh_all, m, po_all, ls, s, it.data(), cv))) return rc;
    conv.assign((size_t)s, 1);
    for (int k = 0; k < s; ++k) {
        iters[(size_t)k] = it[(size_t)k];
        conv[(size_t)k] = cv[k] ? 1 : 0;
        // y_k = the first ell s entries of x_k, into column k of Y
        HIPCHK(copy_strided(Y + k, kBlkRhs * sizeof(double), r.cx + (int64_t)k * m, sizeof(double), sizeof(double),
                                (size_t)ls, hipMemcpyDeviceToDevice, st));
    }
    po_h.assign((size_t)s, ParamOut{});
    HIPCHK(hipMemcpyAsync(po_h.data(), po_all, (size_t)s * sizeof(ParamOut), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MQH_OK;
}

int check_block_args(const mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, int32_t ell) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (F == nullptr) return fail(MQH_EINVAL, "NULL right-hand sides");
    if (nrhs < 1 || nrhs > kBlkRhs) return fail(MQH_EINVAL, "nrhs must be in [1, MQH_BLOCK_RHS]");
    if (ldf < p->n) return fail(MQH_EINVAL, "ldf must be >= n");
    if (ell < 1 || (int64_t)ell * nrhs > p->n || (int64_t)(ell + 1) * nrhs > MQH_BLOCK_MAX_DIM)
        return fail(MQH_EINVAL, "need ell >= 1, ell nrhs <= n and (ell + 1) nrhs <= MQH_BLOCK_MAX_DIM");
    return MQH_OK;
}

// F (n x nrhs, leading dimension ldf, host or device) into W's first block.
int stage_block(mqh_problem* p, BlockWs& b, const double* F, int64_t ldf, int32_t nrhs, uint32_t flags) {
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) {
        for (int32_t k = 0; k < nrhs; ++k)
            if (!all_finite(F + (int64_t)k * ldf, p->n)) return fail(MQH_EINVAL, "non-finite right-hand side");
    }
    HIPCHK(copy_strided(b.W, (size_t)p->ldn * sizeof(double), F, (size_t)ldf * sizeof(double),
                            (size_t)p->n * sizeof(double), (size_t)nrhs, kind_in(flags), p->stream));
    return MQH_OK;
}

}  // namespace

extern "C" {

int mqh_version(void) { return MQH_VERSION; }

const char* mqh_status_str(int status) {
    switch (status) {
        case MQH_OK: return "ok";
        case MQH_EINVAL: return "invalid argument";
        case MQH_ENOMEM: return "out of device memory";
        case MQH_EDEVICE: return "device error";
        case MQH_WBREAKDOWN: return "Golub-Kahan breakdown (fewer steps kept)";
        case MQH_WEDGE: return "parameter at the end of the search grid";
        case MQH_WNOCONV: return "full SVD: Jacobi sweeps stopped at their limit";
        default: return "unknown status";
    }
}

const char* mqh_last_error(void) { return g_last_error.c_str(); }

int64_t mqh_problem_size(const mqh_problem* p) { return p ? p->n : -1; }

int64_t mqh_device_bytes(void) {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    return (int64_t)g_mem_bytes;
}

int mqh_problem_destroy(mqh_problem* p) {
    if (p == nullptr) return MQH_OK;
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    dfree(p->X64);
    dfree(p->X32);
    dfree(p->mlp);
    dfree(p->pout2);
    dfree(p->XS);
    dfree(p->XS64);
    dfree(p->perm);
    dfree(p->iperm);
    dfree(p->frames);
    dfree(p->cf);
    dfree(p->sym_items);
    dfree(p->sym_first);
    dfree(p->sym_row);
    dfree(p->sym_col);
    dfree(p->A);
    dfree(p->pk_tile_base);
    dfree(p->pk_items);
    dfree(p->pk_item_first);
    dfree(p->PR);
    dfree(p->PC);
    dfree(p->vx);
    dfree(p->vy);
    dfree(p->vz);
    dfree(p->W);
    dfree(p->Z);
    dfree(p->alpha);
    dfree(p->beta);
    dfree(p->st);
    dfree(p->gpart);
    dfree(p->cvec);
    dfree(p->npart);
    dfree(p->sv);
    dfree(p->ftil);
    dfree(p->Vw);
    dfree(p->V);
    dfree(p->y);
    dfree(p->pout);
    dfree(p->svd_status);
    dfree(p->coef);
    dfree(p->E);
    dfree(p->EP);
    dfree(p->u);
    multi_free(p->mw);
    block_cache_free(p->bc);
    if (p->hres) (void)hipHostFree(p->hres);
    for (auto& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : p->pev) (void)hipEventDestroy(e);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return MQH_OK;
}

int mqh_problem_create(const double* x_int, int64_t n_int, const double* x_bnd, int64_t n_bnd, double kappa,
                       double eps, int32_t op_mode, void* stream, uint32_t flags, mqh_problem** out) {
    if (out == nullptr) return fail(MQH_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_int < 0 || n_bnd < 0 || n_int + n_bnd <= 0) return fail(MQH_EINVAL, "need n_int >= 0, n_bnd >= 0, n >= 1");
    if (n_int + n_bnd > (int64_t)1 << 31) return fail(MQH_EINVAL, "n too large");
    if ((n_int > 0 && x_int == nullptr) || (n_bnd > 0 && x_bnd == nullptr)) return fail(MQH_EINVAL, "NULL nodes");
    if (!isfinite(kappa) || !isfinite(eps) || !(eps > 0.0)) return fail(MQH_EINVAL, "need finite kappa and eps > 0");
    if (op_mode < MQH_OP_STORED_FP64 || op_mode > MQH_OP_MATFREE_FP32) return fail(MQH_EINVAL, "unknown op_mode");
    const int64_t n = n_int + n_bnd;
    std::vector<double> xyz((size_t)(3 * n));
    if (flags & MQH_FLAG_DEVICE_PTRS) {
        if (n_int) HIPCHK(hipMemcpy(xyz.data(), x_int, (size_t)(3 * n_int) * sizeof(double), hipMemcpyDeviceToHost));
        if (n_bnd)
            HIPCHK(hipMemcpy(xyz.data() + 3 * n_int, x_bnd, (size_t)(3 * n_bnd) * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        if (n_int) memcpy(xyz.data(), x_int, (size_t)(3 * n_int) * sizeof(double));
        if (n_bnd) memcpy(xyz.data() + 3 * n_int, x_bnd, (size_t)(3 * n_bnd) * sizeof(double));
    }
    if (!all_finite(xyz.data(), 3 * n)) return fail(MQH_EINVAL, "non-finite node coordinate");

    mqh_problem* p = new mqh_problem();
    int rc = MQH_OK;
    auto bail = [&](int code) {
        mqh_problem_destroy(p);
        return code;
    };
    HIPCHK(hipGetDevice(&p->device));
    p->n = n;
    p->n_int = n_int;
    p->n_bnd = n_bnd;
    p->ldn = round_up(n, 64);
    p->kappa = kappa;
    p->eps = eps;
    p->mode = op_mode;
    p->fixed_shapes = (flags & MQH_FLAG_FIXED_SHAPES) != 0;
    p->ec.k2 = kappa * kappa;
    p->ec.e2 = eps * eps;
    p->ec.e2x2 = 2.0 * eps * eps;
    p->ec.k2f = (float)p->ec.k2;
    p->ec.e2f = (float)p->ec.e2;
    p->ec.e2x2f = (float)p->ec.e2x2;
    p->d_int = 1.0 / (p->ec.k2 + 3.0 * p->ec.e2);
    p->ec_rs = p->ec;
    p->ec_rs.k2 = p->d_int * p->ec.k2;
    p->ec_rs.e2 = p->d_int * p->ec.e2;
    p->ec_rs.e2x2 = p->d_int * p->ec.e2x2;
    p->ec_rs.k2f = (float)p->ec_rs.k2;
    p->ec_rs.e2f = (float)p->ec_rs.e2;
    p->ec_rs.e2x2f = (float)p->ec_rs.e2x2;
    for (int a = 0; a < 3; ++a) {
        double lo = xyz[a], hi = xyz[a];
        for (int64_t i = 1; i < n; ++i) {
            lo = xyz[3 * i + a] < lo ? xyz[3 * i + a] : lo;
            hi = xyz[3 * i + a] > hi ? xyz[3 * i + a] : hi;
        }
        p->center[a] = 0.5 * (lo + hi);
    }
    if (stream != nullptr) {
        p->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(e, "hipStreamCreate"));
        p->own_stream = true;
    }
    for (auto& e : p->ev)
        if (hipEventCreate(&e) != hipSuccess) return bail(hip_fail(hipErrorUnknown, "hipEventCreate"));
    std::vector<double4> r64((size_t)n);
    std::vector<float4> r32((size_t)n);
    to_records(p, xyz.data(), n, r64.data(), r32.data());
    if ((rc = dalloc(&p->X64, (size_t)n))) return bail(rc);
    if ((rc = dalloc(&p->X32, (size_t)n))) return bail(rc);
    if ((rc = dalloc(&p->vx, (size_t)p->ldn))) return bail(rc);
    if ((rc = dalloc(&p->vy, (size_t)p->ldn))) return bail(rc);
    if ((rc = dalloc(&p->vz, (size_t)p->ldn))) return bail(rc);
    if ((rc = dalloc(&p->st, 1))) return bail(rc);
    if ((rc = dalloc(&p->npart, (size_t)(update_blocks(n) > 1024 ? update_blocks(n) : 1024)))) return bail(rc);
    if ((rc = dalloc(&p->pout, 1))) return bail(rc);
    if ((rc = dalloc(&p->svd_status, 1))) return bail(rc);
    if ((rc = dalloc(&p->coef, (size_t)p->ldn))) return bail(rc);
    {
        hipError_t e = hipHostMalloc((void**)&p->hres, sizeof(HostResults), hipHostMallocDefault);
        if (e != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(p->X64, r64.data(), (size_t)n * sizeof(double4), hipMemcpyHostToDevice, p->stream)) ||
        (e = hipMemcpyAsync(p->X32, r32.data(), (size_t)n * sizeof(float4), hipMemcpyHostToDevice, p->stream)) ||
        (e = hipMemsetAsync(p->vx, 0, (size_t)p->ldn * sizeof(double), p->stream)) ||
        (e = hipMemsetAsync(p->vy, 0, (size_t)p->ldn * sizeof(double), p->stream)) ||
        (e = hipMemsetAsync(p->vz, 0, (size_t)p->ldn * sizeof(double), p->stream)) ||
        (e = hipMemsetAsync(p->coef, 0, (size_t)p->ldn * sizeof(double), p->stream)))
        return bail(hip_fail(e, "upload"));
    if (op_mode == MQH_OP_MATFREE_FP32 || op_mode == MQH_OP_MATFREE_FP64) {
        // both matrix-free modes run over unordered node pairs in the sorted order
        std::vector<int32_t> perm;
        std::vector<float4> rs, frames;
        std::vector<double4> rs64;
        sorted_layout(r64, n, n_int, perm, rs, frames, &rs64);
        if ((rc = dalloc(&p->perm, (size_t)n))) return bail(rc);
        if ((rc = dalloc(&p->iperm, (size_t)n))) return bail(rc);
        std::vector<int32_t> iperm((size_t)n);
        for (int64_t q = 0; q < n; ++q) iperm[(size_t)perm[(size_t)q]] = (int32_t)q;
        if ((e = hipMemcpyAsync(p->perm, perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice,
                                p->stream)) ||
            (e = hipMemcpyAsync(p->iperm, iperm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice,
                                p->stream)))
            return bail(hip_fail(e, "upload of the sorted layout"));
        if (op_mode == MQH_OP_MATFREE_FP32) {
            // nodes are centred, so |P - Q| <= 2 max |P|
            double m2 = 0.0;
            for (const auto& q : rs) {
                const double r2 = (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z;
                m2 = r2 > m2 ? r2 : m2;
            }
            p->blk_tmax = (1.0 + 4.0 * m2) * (1.0 + 1e-3);
            if ((rc = dalloc(&p->XS, (size_t)n)) || (rc = dalloc(&p->frames, frames.size())) ||
                (rc = dalloc(&p->cf, (size_t)n)))
                return bail(rc);
            if ((e = hipMemcpyAsync(p->XS, rs.data(), (size_t)n * sizeof(float4), hipMemcpyHostToDevice,
                                    p->stream)) ||
                (e = hipMemcpyAsync(p->frames, frames.data(), frames.size() * sizeof(float4), hipMemcpyHostToDevice,
                                    p->stream)))
                return bail(hip_fail(e, "upload of the sorted layout"));
        } else {
            if ((rc = dalloc(&p->XS64, (size_t)n))) return bail(rc);
            if ((e = hipMemcpyAsync(p->XS64, rs64.data(), (size_t)n * sizeof(double4), hipMemcpyHostToDevice,
                                    p->stream)))
                return bail(hip_fail(e, "upload of the sorted layout"));
        }
        if ((e = hipStreamSynchronize(p->stream))) return bail(hip_fail(e, "upload of the sorted layout"));
        std::vector<int2> items;
        std::vector<int32_t> first;
        sym_tables(n, n_int, p->sym, items, first);
        if ((rc = dalloc(&p->sym_items, items.size())) || (rc = dalloc(&p->sym_first, first.size())) ||
            (rc = dalloc(&p->sym_row, items.size() * (size_t)p->sym.F * kMfmFixed)) ||
            (rc = dalloc(&p->sym_col, items.size() * (size_t)p->sym.Lb * kMfmFixed)))
            return bail(rc);
        if ((e = hipMemcpyAsync(p->sym_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice,
                                p->stream)) ||
            (e = hipMemcpyAsync(p->sym_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                p->stream)) ||
            (e = hipStreamSynchronize(p->stream)))
            return bail(hip_fail(e, "upload of the pair-product tables"));
        p->sym.items = p->sym_items;
        p->sym.item_first = p->sym_first;
    }
    if (op_mode == MQH_OP_STORED_FP64) {
        PackedTables t;
        packed_tables(n, n_int, t);
        p->pk_max_row = t.max_row;
        p->pk_tiles = t.tile_base[(size_t)t.nt];
        if ((rc = dalloc(&p->pk_tile_base, t.tile_base.size())) || (rc = dalloc(&p->pk_items, t.items.size())) ||
            (rc = dalloc(&p->pk_item_first, t.item_first.size())) ||
            (rc = dalloc(&p->PR, t.items.size() * (size_t)kTile)) ||
            (rc = dalloc(&p->PC, (size_t)p->pk_tiles * (size_t)kTile)) ||
            (rc = dalloc(&p->A, (size_t)p->pk_tiles * (size_t)kTileElems)))
            return bail(rc);
        p->pk.n = n;
        p->pk.n_int = n_int;
        p->pk.nti = t.nti;
        p->pk.nt = t.nt;
        p->pk.nitems = (int32_t)t.items.size();
        p->pk.pad = 0;
        p->pk.tile_base = p->pk_tile_base;
        p->pk.items = p->pk_items;
        p->pk.item_first = p->pk_item_first;
        if ((e = hipMemcpyAsync(p->pk_tile_base, t.tile_base.data(), t.tile_base.size() * sizeof(int64_t),
                                hipMemcpyHostToDevice, p->stream)) ||
            (e = hipMemcpyAsync(p->pk_items, t.items.data(), t.items.size() * sizeof(int4), hipMemcpyHostToDevice,
                                p->stream)) ||
            (e = hipMemcpyAsync(p->pk_item_first, t.item_first.data(), t.item_first.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, p->stream)))
            return bail(hip_fail(e, "upload of the tile tables"));
        launch_assemble_packed(p->X64, p->pk, p->pk_max_row, p->ec, p->A, p->stream);
        if ((e = hipGetLastError())) return bail(hip_fail(e, "assembly launch"));
        // the tables must stay alive until the copies have run
        if ((e = hipStreamSynchronize(p->stream))) return bail(hip_fail(e, "assembly"));
    }
    if ((e = hipStreamSynchronize(p->stream))) return bail(hip_fail(e, "create"));
    *out = p;
    return MQH_OK;
}

int mqh_apply(mqh_problem* p, int32_t trans, const double* x, double shift, const double* z, double* y, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (x == nullptr || y == nullptr) return fail(MQH_EINVAL, "NULL vector");
    if (trans != 0 && trans != 1) return fail(MQH_EINVAL, "trans must be 0 or 1");
    if (!isfinite(shift)) return fail(MQH_EINVAL, "non-finite shift");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, (flags & MQH_FLAG_ROW_SCALE) ? 1 : 0))) return rc;
    if ((rc = stage_in(p->vx, x, p->n, flags, p->stream))) return rc;
    if (z && (rc = stage_in(p->vz, z, p->n, flags, p->stream))) return rc;
    if ((rc = op_product(p, trans, p->vx, nullptr, shift, z ? p->vz : nullptr, p->vy, nullptr, false))) return rc;
    HIPCHK(hipMemcpyAsync(y, p->vy, (size_t)p->n * sizeof(double), kind_out(flags), p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return MQH_OK;
}

int mqh_matrix_rows(mqh_problem* p, int64_t row0, int64_t count, double* out, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (out == nullptr || row0 < 0 || count < 1 || row0 + count > p->n) return fail(MQH_EINVAL, "bad row range");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, (flags & MQH_FLAG_ROW_SCALE) ? 1 : 0))) return rc;
    const bool dev = (flags & MQH_FLAG_DEVICE_PTRS) != 0;
    const int64_t chunk = 1024;
    double* tmp = nullptr;
    if (!dev && (rc = dalloc(&tmp, (size_t)(chunk * p->n)))) return rc;
    for (int64_t r = row0; r < row0 + count; r += chunk) {
        const int64_t c = (row0 + count - r) < chunk ? (row0 + count - r) : chunk;
        double* dst = dev ? out + (r - row0) * p->n : tmp;
        hipError_t e;
        if (p->mode == MQH_OP_STORED_FP64) {
            launch_packed_rows(p->A, p->pk, r, c, dst, p->stream);
            e = hipGetLastError();
        } else {
            launch_gen_rows(p->mode == MQH_OP_MATFREE_FP64 ? 64 : 32,
                            p->mode == MQH_OP_MATFREE_FP64 ? (const void*)p->X64 : (const void*)p->X32, p->n, p->n_int,
                            r, c, op_ec(p), dst, p->stream);
            e = hipGetLastError();
        }
        if (e == hipSuccess && !dev)
            e = hipMemcpyAsync(out + (r - row0) * p->n, tmp, (size_t)(c * p->n) * sizeof(double), hipMemcpyDeviceToHost,
                               p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) {
            dfree(tmp);
            return hip_fail(e, "matrix rows");
        }
    }
    dfree(tmp);
    return MQH_OK;
}

int mqh_gkb(mqh_problem* p, const double* f, int32_t ell, int32_t reorth, double* W, double* Z, double* alpha,
            double* beta, int32_t* ell_done, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (f == nullptr) return fail(MQH_EINVAL, "NULL f");
    if (ell < 1 || ell > p->n || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= min(n, MQH_MAX_ELL)");
    if (reorth != 0 && reorth != 1) return fail(MQH_EINVAL, "reorth must be 0 or 1");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, (flags & MQH_FLAG_ROW_SCALE) ? 1 : 0))) return rc;
    if ((rc = ensure_gkb(p, ell))) return rc;
    if ((rc = stage_in(p->vx, f, p->n, flags, p->stream))) return rc;
    if ((rc = scale_rhs(p, p->vx, 1, 0))) return rc;
    if ((rc = run_gkb(p, ell, reorth, false))) return rc;
    HIPCHK(hipMemcpyAsync(&p->hres->st, p->st, sizeof(GkbState), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    double b1 = 0.0;
    HIPCHK(hipMemcpy(&b1, p->beta, sizeof(double), hipMemcpyDeviceToHost));
    if (!isfinite(b1)) return fail(MQH_EINVAL, "non-finite right-hand side");
    const int32_t done = p->hres->st.ell_done;
    const hipMemcpyKind ko = kind_out(flags);
    const int64_t n = p->n;
    // columns past the kept steps are zero in the outputs
    auto copy_cols = [&](double* dst, const double* src, int32_t total, int32_t valid) -> int {
        if (dst == nullptr) return MQH_OK;
        if (valid > 0)
            HIPCHK(copy_strided(dst, (size_t)n * sizeof(double), src, (size_t)p->ldn * sizeof(double),
                                    (size_t)n * sizeof(double), (size_t)valid, ko, p->stream));
        if (total > valid) {
            if (flags & MQH_FLAG_DEVICE_PTRS) {
                launch_fill(dst + (int64_t)valid * n, (int64_t)(total - valid) * n, 0.0, p->stream);
                LAUNCHCHK("fill");
            } else {
                memset(dst + (int64_t)valid * n, 0, (size_t)(total - valid) * n * sizeof(double));
            }
        }
        return MQH_OK;
    };
    const int32_t wcols = p->hres->st.flag == 2 ? done : done + 1;  // w_{done+1} is zero after a beta breakdown
    if ((rc = copy_cols(W, p->W, ell + 1, wcols))) return rc;
    if ((rc = copy_cols(Z, p->Z, ell, done))) return rc;
    if (alpha) HIPCHK(hipMemcpyAsync(alpha, p->alpha, (size_t)ell * sizeof(double), ko, p->stream));
    if (beta) HIPCHK(hipMemcpyAsync(beta, p->beta, (size_t)(ell + 1) * sizeof(double), ko, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    if (ell_done) *ell_done = done;
    return (done < ell || p->hres->st.flag != 0) ? MQH_WBREAKDOWN : MQH_OK;
}

int mqh_solve(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts, double* coef,
              double* gkb_alpha, double* gkb_beta, double* ritz_sv, mqh_solve_info* info) {
    clear_info(info);
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (opts == nullptr) return fail(MQH_EINVAL, "NULL opts");
    if (coef == nullptr) return fail(MQH_EINVAL, "NULL coef");
    if ((p->n_int > 0 && f_int == nullptr) || (p->n_bnd > 0 && g_bnd == nullptr)) return fail(MQH_EINVAL, "NULL data");
    if ((rc = check_opts(p, opts))) return rc;
    const int32_t ell = opts->ell;
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    const uint32_t flags = opts->flags;
    const bool timed = (flags & MQH_FLAG_TIME_PRODUCTS) != 0;
    HIPCHK(hipSetDevice(p->device));
    hipStream_t s = p->stream;
    if ((rc = ensure_gkb(p, ell))) return rc;
    if ((rc = set_row_scale(p, opts->row_scale))) return rc;
    for (auto& e : p->pev) (void)hipEventDestroy(e);
    p->pev.clear();
    if (timed) p->pev.reserve((size_t)ell * 4);
    HIPCHK(hipEventRecord(p->ev[0], s));
    if ((rc = stage_in(p->vx, f_int, p->n_int, flags, s))) return rc;
    if ((rc = stage_in(p->vx + p->n_int, g_bnd, p->n_bnd, flags, s))) return rc;
    if ((rc = scale_rhs(p, p->vx, 1, 0))) return rc;
    HIPCHK(hipEventRecord(p->ev[1], s));
    if ((rc = run_gkb(p, ell, opts->reorth, timed))) return rc;
    HIPCHK(hipEventRecord(p->ev[2], s));
    const int32_t* lp = &p->st->ell_done;
    const bool lsqr = opts->method == MQH_METHOD_LSQR;
    const bool svd_runs = !lsqr || ritz_sv != nullptr;
    launch_fill(p->sv, ell, 0.0, s);
    if (svd_runs) {
        launch_bidiag_svd(p->alpha, p->beta, ell, lp, p->Vw, p->sv, p->ftil, p->V, ell, p->svd_status, 0, s);
        LAUNCHCHK("projected SVD");
    }
    HIPCHK(hipEventRecord(p->ev[3], s));
    if (lsqr) {
        launch_lsqr(p->alpha, p->beta, ell, lp, p->n, opts->rule, opts->k_trunc, nullptr, nullptr, p->pout, p->y, ell,
                    s);
    } else {
        launch_param_choice(p->sv, p->ftil, ell, lp, opts->method, opts->rule, J, opts->lambda_fixed, opts->k_trunc,
                            opts->gcv_weight, nullptr, p->pout, s);
        launch_proj_solution(p->sv, p->ftil, p->V, ell, ell, lp, opts->method, 0.0, 0, p->pout, p->y, ell, s);
    }
    LAUNCHCHK("parameter choice");
    HIPCHK(hipEventRecord(p->ev[4], s));
    launch_lift(p->Z, p->ldn, p->n, ell, lp, p->y, p->coef, s);
    LAUNCHCHK("lift");
    HIPCHK(hipEventRecord(p->ev[5], s));
    HIPCHK(hipMemcpyAsync(&p->hres->st, p->st, sizeof(GkbState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&p->hres->po, p->pout, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&p->hres->svd_status, p->svd_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double b1 = 0.0;
    HIPCHK(hipMemcpy(&b1, p->beta, sizeof(double), hipMemcpyDeviceToHost));
    if (!isfinite(b1)) return fail(MQH_EINVAL, "non-finite right-hand side");
    if (svd_runs && p->hres->svd_status < 0) return fail(MQH_EDEVICE, "projected SVD did not converge");
    const hipMemcpyKind ko = kind_out(flags);
    HIPCHK(hipMemcpyAsync(coef, p->coef, (size_t)p->n * sizeof(double), ko, s));
    if (gkb_alpha) HIPCHK(hipMemcpyAsync(gkb_alpha, p->alpha, (size_t)ell * sizeof(double), ko, s));
    if (gkb_beta) HIPCHK(hipMemcpyAsync(gkb_beta, p->beta, (size_t)(ell + 1) * sizeof(double), ko, s));
    if (ritz_sv) HIPCHK(hipMemcpyAsync(ritz_sv, p->sv, (size_t)ell * sizeof(double), ko, s));
    HIPCHK(hipEventRecord(p->ev[6], s));
    HIPCHK(hipStreamSynchronize(s));
    const GkbState& st = p->hres->st;
    const ParamOut& po = p->hres->po;
    uint32_t iflags = po.flags;
    if (st.flag != 0) iflags |= MQH_INFO_BREAKDOWN;
    if (svd_runs && p->hres->svd_status == 1) iflags |= MQH_INFO_SVD_QR;
    if (info) {
        info->ell_done = st.ell_done;
        info->k_chosen = po.k;
        info->lambda_chosen = po.lambda;
        info->crit = po.crit;
        info->resid_norm = po.rho;
        info->sol_norm = po.eta;
        info->flags = iflags;
        float ms = 0.f;
        const int pairs[6][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {0, 6}};
        for (int q = 0; q < 6; ++q) {
            if (hipEventElapsedTime(&ms, p->ev[pairs[q][0]], p->ev[pairs[q][1]]) == hipSuccess) info->t_ms[q] = ms;
        }
        if (timed) {
            // products alternate A^T (even pairs) and A (odd pairs)
            double tt = 0.0, ta = 0.0;
            for (size_t q = 0; q + 1 < p->pev.size(); q += 2)
                if (hipEventElapsedTime(&ms, p->pev[q], p->pev[q + 1]) == hipSuccess) ((q / 2) % 2 == 0 ? tt : ta) += ms;
            info->t_ms[6] = tt;
            info->t_ms[7] = ta;
        }
    }
    if (st.flag != 0) return MQH_WBREAKDOWN;
    if (iflags & (MQH_INFO_GCV_AT_EDGE | MQH_INFO_LCURVE_AT_EDGE)) return MQH_WEDGE;
    return MQH_OK;
}

int mqh_apply_multi(mqh_problem* p, int32_t trans, const double* X, int64_t ldx, int32_t nrhs, const double* shifts,
                    const double* Zs, int64_t ldz, double* Y, int64_t ldy, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (X == nullptr || Y == nullptr) return fail(MQH_EINVAL, "NULL X or Y");
    if (trans != 0 && trans != 1) return fail(MQH_EINVAL, "trans must be 0 or 1");
    if (nrhs < 1) return fail(MQH_EINVAL, "need nrhs >= 1");
    if (ldx < p->n || ldy < p->n || (Zs != nullptr && ldz < p->n))
        return fail(MQH_EINVAL, "need leading dimensions >= n");
    if (shifts != nullptr)
        for (int32_t k = 0; k < nrhs; ++k)
            if (!isfinite(shifts[k])) return fail(MQH_EINVAL, "non-finite shift");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, (flags & MQH_FLAG_ROW_SCALE) ? 1 : 0))) return rc;
    hipStream_t s = p->stream;
    for (int k0 = 0; k0 < nrhs; k0 += kBlkRhs) {
        const int nz = nrhs - k0 < kBlkRhs ? nrhs - k0 : kBlkRhs;
        if ((rc = ensure_multi(p, nz, 1))) return rc;
        MultiWs& w = p->mw;
        if ((rc = stage_multi(p, X, ldx, k0, nz, flags))) return rc;
        const double* zs = nullptr;
        if (Zs != nullptr) {
            if (!(flags & MQH_FLAG_DEVICE_PTRS))
                for (int k = 0; k < nz; ++k)
                    if (!all_finite(Zs + (int64_t)(k0 + k) * ldz, p->n)) return fail(MQH_EINVAL, "non-finite z");
            HIPCHK(copy_strided(w.Z, (size_t)w.bstr * sizeof(double), Zs + (int64_t)k0 * ldz,
                                    (size_t)ldz * sizeof(double), (size_t)p->n * sizeof(double), (size_t)nz,
                                    kind_in(flags), s));
            zs = w.Z;
        }
        // the shifts go in column 0 of the run's alpha
        std::vector<double> sh((size_t)nz * (size_t)w.vstr, 0.0);
        if (shifts != nullptr)
            for (int k = 0; k < nz; ++k) sh[(size_t)k * (size_t)w.vstr] = shifts[k0 + k];
        HIPCHK(hipMemcpyAsync(w.alpha, sh.data(), sh.size() * sizeof(double), hipMemcpyHostToDevice, s));
        if ((rc = block_product(p, nz, trans, w.X, p->ldn, w.alpha, w.vstr, zs, w.bstr, w.Y, nullptr, false, false,
                                false)))
            return rc;
        HIPCHK(copy_strided(Y + (int64_t)k0 * ldy, (size_t)ldy * sizeof(double), w.Y,
                                (size_t)p->ldn * sizeof(double), (size_t)p->n * sizeof(double), (size_t)nz,
                                kind_out(flags), s));
        HIPCHK(hipStreamSynchronize(s));  // sh lives until the copy has run
    }
    return MQH_OK;
}

int mqh_gkb_multi(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, int32_t ell, int32_t reorth, double* W,
                  double* Z, double* alpha, double* beta, int32_t* ell_done, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (F == nullptr) return fail(MQH_EINVAL, "NULL F");
    if (nrhs < 1) return fail(MQH_EINVAL, "need nrhs >= 1");
    if (ldf < p->n) return fail(MQH_EINVAL, "need ldf >= n");
    if (ell < 1 || ell > p->n || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= min(n, MQH_MAX_ELL)");
    if (reorth != 0 && reorth != 1) return fail(MQH_EINVAL, "reorth must be 0 or 1");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, (flags & MQH_FLAG_ROW_SCALE) ? 1 : 0))) return rc;
    hipStream_t s = p->stream;
    const int64_t n = p->n;
    const hipMemcpyKind ko = kind_out(flags);
    const bool dev = (flags & MQH_FLAG_DEVICE_PTRS) != 0;
    bool broke = false;
    for (int k0 = 0; k0 < nrhs; k0 += kBlkRhs) {
        const int nz = nrhs - k0 < kBlkRhs ? nrhs - k0 : kBlkRhs;
        if ((rc = ensure_multi(p, nz, ell))) return rc;
        MultiWs& w = p->mw;
        if ((rc = stage_multi(p, F, ldf, k0, nz, flags))) return rc;
        if ((rc = scale_rhs(p, w.X, nz, p->ldn))) return rc;
        if ((rc = run_gkb_multi(p, nz, ell, reorth, false))) return rc;
        std::vector<GkbState> st((size_t)nz);
        std::vector<double> b1((size_t)nz);
        HIPCHK(hipMemcpyAsync(st.data(), w.st, (size_t)nz * sizeof(GkbState), hipMemcpyDeviceToHost, s));
        HIPCHK(copy_strided(b1.data(), sizeof(double), w.beta, (size_t)w.vstr * sizeof(double), sizeof(double),
                                (size_t)nz, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < nz; ++k)
            if (!isfinite(b1[(size_t)k])) return fail(MQH_EINVAL, "non-finite right-hand side");
        for (int k = 0; k < nz; ++k) {
            const int64_t r = k0 + k;
            const int32_t done = st[(size_t)k].ell_done;
            broke = broke || done < ell || st[(size_t)k].flag != 0;
            auto copy_cols = [&](double* dst, const double* src, int32_t total, int32_t valid) -> int {
                if (dst == nullptr) return MQH_OK;
                if (valid > 0)
                    HIPCHK(copy_strided(dst, (size_t)n * sizeof(double), src, (size_t)p->ldn * sizeof(double),
                                            (size_t)n * sizeof(double), (size_t)valid, ko, s));
                if (total > valid) {
                    if (dev) {
                        launch_fill(dst + (int64_t)valid * n, (int64_t)(total - valid) * n, 0.0, s);
                        LAUNCHCHK("fill");
                    } else {
                        memset(dst + (int64_t)valid * n, 0, (size_t)(total - valid) * n * sizeof(double));
                    }
                }
                return MQH_OK;
            };
            const int32_t wcols = st[(size_t)k].flag == 2 ? done : done + 1;
            if ((rc = copy_cols(W ? W + r * (ell + 1) * n : nullptr, w.W + k * w.bstr, ell + 1, wcols))) return rc;
            if ((rc = copy_cols(Z ? Z + r * ell * n : nullptr, w.Z + k * w.bstr, ell, done))) return rc;
            if (alpha)
                HIPCHK(hipMemcpyAsync(alpha + r * ell, w.alpha + k * w.vstr, (size_t)ell * sizeof(double), ko, s));
            if (beta)
                HIPCHK(hipMemcpyAsync(beta + r * (ell + 1), w.beta + k * w.vstr, (size_t)(ell + 1) * sizeof(double),
                                      ko, s));
            if (ell_done) ell_done[r] = done;
        }
        HIPCHK(hipStreamSynchronize(s));
    }
    return broke ? MQH_WBREAKDOWN : MQH_OK;
}

int mqh_solve_multi(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, const mqh_solve_opts* opts,
                    double* coef, int64_t ldc, mqh_solve_info* info) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (opts == nullptr) return fail(MQH_EINVAL, "NULL opts");
    if (F == nullptr || coef == nullptr) return fail(MQH_EINVAL, "NULL F or coef");
    if (nrhs < 1) return fail(MQH_EINVAL, "need nrhs >= 1");
    if (ldf < p->n || ldc < p->n) return fail(MQH_EINVAL, "need ldf >= n and ldc >= n");
    if (info)
        for (int32_t k = 0; k < nrhs; ++k) clear_info(info + k);
    if ((rc = check_opts(p, opts))) return rc;
    const int32_t ell = opts->ell;
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    const uint32_t flags = opts->flags;
    const bool timed = (flags & MQH_FLAG_TIME_PRODUCTS) != 0;
    const bool lsqr = opts->method == MQH_METHOD_LSQR;
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, opts->row_scale))) return rc;
    hipStream_t s = p->stream;
    const hipMemcpyKind ko = kind_out(flags);
    bool broke = false, edge = false;
    for (int k0 = 0; k0 < nrhs; k0 += kBlkRhs) {
        const int nz = nrhs - k0 < kBlkRhs ? nrhs - k0 : kBlkRhs;
        if ((rc = ensure_multi(p, nz, ell))) return rc;
        MultiWs& w = p->mw;
        for (auto& e : p->pev) (void)hipEventDestroy(e);
        p->pev.clear();
        if (timed) p->pev.reserve((size_t)ell * 4 * (size_t)nz);
        HIPCHK(hipEventRecord(p->ev[0], s));
        if ((rc = stage_multi(p, F, ldf, k0, nz, flags))) return rc;
        if ((rc = scale_rhs(p, w.X, nz, p->ldn))) return rc;
        HIPCHK(hipEventRecord(p->ev[1], s));
        if ((flags & MQH_FLAG_GRAPH) && !timed) {
            if ((rc = run_gkb_multi_graph(p, nz, ell, opts->reorth))) return rc;
        } else {
            if ((rc = run_gkb_multi(p, nz, ell, opts->reorth, timed))) return rc;
        }
        HIPCHK(hipEventRecord(p->ev[2], s));
        const int32_t* lp = &w.st->ell_done;
        const ProjBatch pb{w.vstr, (int64_t)w.ell_cap * w.ell_cap, (int64_t)(sizeof(GkbState) / sizeof(int32_t)), 0,
                           (int64_t)svd_ws_doubles(w.ell_cap)};
        launch_fill(w.sv, (int64_t)nz * w.vstr, 0.0, s);
        if (!lsqr) {
            launch_bidiag_svd(w.alpha, w.beta, ell, lp, w.Vw, w.sv, w.ftil, w.V, ell, w.status, 0, s, nz, pb);
            LAUNCHCHK("projected SVD");
        }
        HIPCHK(hipEventRecord(p->ev[3], s));
        if (lsqr) {
            launch_lsqr(w.alpha, w.beta, ell, lp, p->n, opts->rule, opts->k_trunc, nullptr, nullptr, w.pout, w.y, ell,
                        s, nz, pb);
        } else {
            launch_param_choice(w.sv, w.ftil, ell, lp, opts->method, opts->rule, J, opts->lambda_fixed, opts->k_trunc,
                                opts->gcv_weight, nullptr, w.pout, s, nz, pb);
            launch_proj_solution(w.sv, w.ftil, w.V, ell, ell, lp, opts->method, 0.0, 0, w.pout, w.y, ell, s, nz, pb);
        }
        LAUNCHCHK("parameter choice");
        HIPCHK(hipEventRecord(p->ev[4], s));
        launch_lift(w.Z, p->ldn, p->n, ell, lp, w.y, w.coef, s, nz,
                    Bz{w.bstr, w.vstr, p->ldn, (int64_t)(sizeof(GkbState) / sizeof(int32_t))});
        LAUNCHCHK("lift");
        HIPCHK(hipEventRecord(p->ev[5], s));
        std::vector<GkbState> st((size_t)nz);
        std::vector<ParamOut> po((size_t)nz);
        std::vector<int32_t> svs((size_t)nz, 0);
        std::vector<double> b1((size_t)nz);
        HIPCHK(hipMemcpyAsync(st.data(), w.st, (size_t)nz * sizeof(GkbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(po.data(), w.pout, (size_t)nz * sizeof(ParamOut), hipMemcpyDeviceToHost, s));
        if (!lsqr) HIPCHK(hipMemcpyAsync(svs.data(), w.status, (size_t)nz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(copy_strided(b1.data(), sizeof(double), w.beta, (size_t)w.vstr * sizeof(double), sizeof(double),
                                (size_t)nz, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < nz; ++k) {
            if (!isfinite(b1[(size_t)k])) return fail(MQH_EINVAL, "non-finite right-hand side");
            if (svs[(size_t)k] < 0) return fail(MQH_EDEVICE, "projected SVD did not converge");
        }
        HIPCHK(copy_strided(coef + (int64_t)k0 * ldc, (size_t)ldc * sizeof(double), w.coef,
                                (size_t)p->ldn * sizeof(double), (size_t)p->n * sizeof(double), (size_t)nz, ko, s));
        HIPCHK(hipEventRecord(p->ev[6], s));
        HIPCHK(hipStreamSynchronize(s));
        float t_ms[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        {
            float ms = 0.f;
            const int pairs[6][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {0, 6}};
            for (int q = 0; q < 6; ++q)
                if (hipEventElapsedTime(&ms, p->ev[pairs[q][0]], p->ev[pairs[q][1]]) == hipSuccess) t_ms[q] = ms;
            if (timed) {
                // products alternate A^T (even pairs) and A (odd pairs) when
                // they are block products; one per run otherwise
                const size_t per = (p->mode == MQH_OP_MATFREE_FP32 && nz >= 2) ? 1 : (size_t)nz;
                for (size_t q = 0; q + 1 < p->pev.size(); q += 2)
                    if (hipEventElapsedTime(&ms, p->pev[q], p->pev[q + 1]) == hipSuccess)
                        t_ms[((q / 2) / per) % 2 == 0 ? 6 : 7] += ms;
            }
        }
        for (int k = 0; k < nz; ++k) {
            const GkbState& g = st[(size_t)k];
            const ParamOut& o = po[(size_t)k];
            uint32_t iflags = o.flags;
            if (g.flag != 0) iflags |= MQH_INFO_BREAKDOWN;
            if (!lsqr && svs[(size_t)k] == 1) iflags |= MQH_INFO_SVD_QR;
            broke = broke || g.flag != 0;
            edge = edge || (iflags & (MQH_INFO_GCV_AT_EDGE | MQH_INFO_LCURVE_AT_EDGE)) != 0;
            if (info) {
                mqh_solve_info* in = info + k0 + k;
                in->ell_done = g.ell_done;
                in->k_chosen = o.k;
                in->lambda_chosen = o.lambda;
                in->crit = o.crit;
                in->resid_norm = o.rho;
                in->sol_norm = o.eta;
                in->flags = iflags;
                for (int q = 0; q < 8; ++q) in->t_ms[q] = t_ms[q];
            }
        }
    }
    if (broke) return MQH_WBREAKDOWN;
    if (edge) return MQH_WEDGE;
    return MQH_OK;
}

int mqh_solve_sweep(mqh_sweep_item* items, int32_t count, const mqh_solve_opts* opts, int32_t workers) {
    if (items == nullptr || count < 1) return fail(MQH_EINVAL, "need items and count >= 1");
    if (opts == nullptr) return fail(MQH_EINVAL, "NULL opts");
    for (int32_t k = 0; k < count; ++k) {
        items[k].status = MQH_EINVAL;
        if (items[k].p == nullptr) return fail(MQH_EINVAL, "NULL problem in the sweep");
        for (int32_t q = 0; q < k; ++q)
            if (items[q].p == items[k].p) return fail(MQH_EINVAL, "a problem appears twice in the sweep");
    }
    if (workers < 1) workers = 1;
    if (workers > count) workers = count;
    std::atomic<int32_t> next{0};
    std::mutex mu;
    std::string first_error;
    int first_code = MQH_OK;
    auto work = [&]() {
        for (;;) {
            const int32_t k = next.fetch_add(1);
            if (k >= count) return;
            mqh_sweep_item& it = items[k];
            it.status = mqh_solve_multi(it.p, it.F, it.ldf, it.nrhs, opts, it.coef, it.ldc, it.info);
            if (it.status < 0) {
                std::lock_guard<std::mutex> lock(mu);
                if (first_code == MQH_OK) {
                    first_code = it.status;
                    first_error = g_last_error;
                }
            }
        }
    };
    std::vector<std::thread> pool;
    pool.reserve((size_t)workers - 1);
    for (int32_t t = 1; t < workers; ++t) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    if (first_code != MQH_OK) return fail(first_code, first_error);
    int worst = MQH_OK;
    for (int32_t k = 0; k < count; ++k)
        if (items[k].status == MQH_WBREAKDOWN || (items[k].status == MQH_WEDGE && worst == MQH_OK)) worst = items[k].status;
    return worst;
}

int mqh_full_svd(mqh_problem* p, const double* f, double* sv, double* fhat, int32_t* sweeps, double* off,
                 uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (sv == nullptr) return fail(MQH_EINVAL, "NULL sv");
    if (p->n > MQH_FULL_MAX_N) return fail(MQH_EINVAL, "the full SVD takes n <= MQH_FULL_MAX_N");
    HIPCHK(hipSetDevice(p->device));
    hipStream_t s = p->stream;
    FullRun r;
    if (f != nullptr) {
        if ((rc = dalloc(&r.f, (size_t)p->n))) return rc;
        if ((rc = stage_in(r.f, f, p->n, flags, s))) return rc;
    }
    HIPCHK(hipEventRecord(p->ev[0], s));
    if ((rc = full_svd_run(p, r))) return rc;
    const hipMemcpyKind ko = kind_out(flags);
    HIPCHK(hipMemcpyAsync(sv, r.sv, (size_t)p->n * sizeof(double), ko, s));
    if (fhat) HIPCHK(hipMemcpyAsync(fhat, r.fs, (size_t)p->n * sizeof(double), ko, s));
    HIPCHK(hipStreamSynchronize(s));
    if (sweeps) *sweeps = r.sweeps;
    if (off) *off = r.final_off;
    return r.final_off > full_floor(p->n) ? MQH_WNOCONV : MQH_OK;
}

int mqh_full_solve(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts, double* coef,
                   double* sv, mqh_solve_info* info) {
    clear_info(info);
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (opts == nullptr) return fail(MQH_EINVAL, "NULL opts");
    if (coef == nullptr) return fail(MQH_EINVAL, "NULL coef");
    if ((p->n_int > 0 && f_int == nullptr) || (p->n_bnd > 0 && g_bnd == nullptr)) return fail(MQH_EINVAL, "NULL data");
    if (p->n > MQH_FULL_MAX_N) return fail(MQH_EINVAL, "the full SVD takes n <= MQH_FULL_MAX_N");
    if (opts->row_scale != 0) return fail(MQH_EINVAL, "the full-SVD solve takes row_scale = 0");
    if (opts->method != MQH_METHOD_HKT && opts->method != MQH_METHOD_INE_TSVD)
        return fail(MQH_EINVAL, "method: MQH_METHOD_HKT (Tikhonov filter) or MQH_METHOD_INE_TSVD (TSVD filter)");
    if (opts->rule != MQH_RULE_GCV && opts->rule != MQH_RULE_FIXED)
        return fail(MQH_EINVAL, "rule: MQH_RULE_GCV or MQH_RULE_FIXED");
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    if (J < 3 || J > kMaxGrid) return fail(MQH_EINVAL, "n_grid must be 0 or in [3, 4096]");
    const bool tikh = opts->method == MQH_METHOD_HKT;
    if (tikh && opts->rule == MQH_RULE_FIXED && (!isfinite(opts->lambda_fixed) || opts->lambda_fixed < 0.0))
        return fail(MQH_EINVAL, "lambda_fixed must be finite and >= 0");
    if (!tikh && opts->rule == MQH_RULE_FIXED && (opts->k_trunc < 1 || opts->k_trunc > p->n))
        return fail(MQH_EINVAL, "k_trunc must be in [1, n]");
    const uint32_t flags = opts->flags;
    HIPCHK(hipSetDevice(p->device));
    hipStream_t s = p->stream;
    FullRun r;
    if ((rc = dalloc(&r.f, (size_t)p->n))) return rc;
    if ((rc = stage_in(r.f, f_int, p->n_int, flags, s))) return rc;
    if ((rc = stage_in(r.f + p->n_int, g_bnd, p->n_bnd, flags, s))) return rc;
    HIPCHK(hipEventRecord(p->ev[0], s));
    // ||f||^2 for s_perp (on the host from the staged copy: one read of n values)
    std::vector<double> fh((size_t)p->n);
    HIPCHK(hipMemcpyAsync(fh.data(), r.f, (size_t)p->n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double fn2 = 0.0;
    for (double v : fh) fn2 += v * v;
    if (!isfinite(fn2)) return fail(MQH_EINVAL, "non-finite right-hand side");
    if ((rc = full_svd_run(p, r))) return rc;
    if ((rc = dalloc(&r.fn2, 1))) return rc;
    HIPCHK(hipMemcpyAsync(r.fn2, &fn2, sizeof(double), hipMemcpyHostToDevice, s));
    launch_full_param(r.sv, r.fs, p->n, p->n, r.fn2, p->n, tikh ? 1 : 0, opts->rule == MQH_RULE_FIXED ? 2 : 0, J,
                      opts->lambda_fixed, opts->k_trunc, r.tail, r.po, 1, s);
    LAUNCHCHK("full problem: parameter choice");
    HIPCHK(hipEventRecord(p->ev[4], s));
    int cg_iters = 0;
    bool cg_conv = true;
    if ((rc = full_solution(s, r, p->n, tikh ? 1 : 0, r.fh, p->n, r.po, p->n, 1, &cg_iters, &cg_conv))) return rc;
    HIPCHK(hipEventRecord(p->ev[5], s));
    ParamOut po;
    HIPCHK(hipMemcpyAsync(&po, r.po, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    const hipMemcpyKind ko = kind_out(flags);
    HIPCHK(hipMemcpyAsync(coef, r.cx, (size_t)p->n * sizeof(double), ko, s));
    if (sv) HIPCHK(hipMemcpyAsync(sv, r.sv, (size_t)p->n * sizeof(double), ko, s));
    HIPCHK(hipEventRecord(p->ev[6], s));
    HIPCHK(hipStreamSynchronize(s));
    const bool noconv = r.final_off > full_floor(p->n);
    if (info) {
        info->ell_done = r.sweeps;
        info->k_chosen = po.k;
        info->lambda_chosen = po.lambda;
        info->crit = po.crit;
        info->resid_norm = po.rho;
        info->sol_norm = po.eta;
        info->flags = po.flags | (cg_conv ? 0u : MQH_INFO_SOLVE_NOCONV);
        float ms = 0.f;
        const int pairs[6][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {0, 6}};
        for (int q = 0; q < 6; ++q)
            if (hipEventElapsedTime(&ms, p->ev[pairs[q][0]], p->ev[pairs[q][1]]) == hipSuccess) info->t_ms[q] = ms;
        info->t_ms[6] = (float)r.final_off;
        info->t_ms[7] = cg_iters;
    }
    if (noconv || !cg_conv) return MQH_WNOCONV;
    if (po.flags & MQH_INFO_GCV_AT_EDGE) return MQH_WEDGE;
    return MQH_OK;
}

int mqh_gkb_block(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, int32_t ell, double* C, double* E1,
                  double* W, double* Z, int32_t* ell_done, int32_t* flag, uint32_t flags) {
    if (ell_done) *ell_done = 0;
    if (flag) *flag = 0;
    int rc;
    if ((rc = check_block_args(p, F, ldf, nrhs, ell))) return rc;
    if (C == nullptr) return fail(MQH_EINVAL, "NULL C");
    if (flags & MQH_FLAG_ROW_SCALE) return fail(MQH_EINVAL, "the block Golub-Kahan calls run on A (no row scaling)");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, 0))) return rc;
    hipStream_t st = p->stream;
    if (p->mode == MQH_OP_MATFREE_FP32 && nrhs >= 2 && (rc = ensure_multi(p, nrhs, 1))) return rc;
    BlockWs* bw = nullptr;
    if ((rc = block_ws(p, nrhs, ell, &bw))) return rc;
    BlockWs& b = *bw;
    if ((rc = stage_block(p, b, F, ldf, nrhs, flags))) return rc;
    std::vector<double> Ch;
    double E1h[kBlkRhs * kBlkRhs];
    int32_t ld = 0, fl = 0;
    if ((rc = run_gkb_block(p, b, nrhs, ell, Ch, E1h, &ld, &fl))) return rc;
    const hipMemcpyKind ko = kind_out(flags);
    const int64_t n = p->n, ldn = p->ldn;
    HIPCHK(hipMemcpyAsync(C, Ch.data(), Ch.size() * sizeof(double),
                          (flags & MQH_FLAG_DEVICE_PTRS) ? hipMemcpyHostToDevice : hipMemcpyHostToHost, st));
    if (E1)
        HIPCHK(hipMemcpyAsync(E1, E1h, (size_t)nrhs * nrhs * sizeof(double),
                              (flags & MQH_FLAG_DEVICE_PTRS) ? hipMemcpyHostToDevice : hipMemcpyHostToHost, st));
    if (W)
        HIPCHK(copy_strided(W, (size_t)n * sizeof(double), b.W, (size_t)ldn * sizeof(double), (size_t)n * sizeof(double),
                                (size_t)(ell + 1) * nrhs, ko, st));
    if (Z)
        HIPCHK(copy_strided(Z, (size_t)n * sizeof(double), b.Z, (size_t)ldn * sizeof(double), (size_t)n * sizeof(double),
                                (size_t)ell * nrhs, ko, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ell_done) *ell_done = ld;
    if (flag) *flag = fl;
    return fl ? MQH_WBREAKDOWN : MQH_OK;
}

int mqh_solve_block(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, const mqh_solve_opts* opts,
                    double* coef, int64_t ldc, double* sv, mqh_solve_info* info) {
    if (info && nrhs > 0 && nrhs <= kBlkRhs)
        for (int32_t k = 0; k < nrhs; ++k) clear_info(info + k);
    int rc;
    if (opts == nullptr) return fail(MQH_EINVAL, "NULL opts");
    if ((rc = check_block_args(p, F, ldf, nrhs, opts->ell))) return rc;
    if (coef == nullptr || ldc < p->n) return fail(MQH_EINVAL, "coef must be n x nrhs with ldc >= n");
    if (opts->method != MQH_METHOD_HKT) return fail(MQH_EINVAL, "block solves use MQH_METHOD_HKT (the Tikhonov filter)");
    if (opts->rule != MQH_RULE_GCV && opts->rule != MQH_RULE_FIXED)
        return fail(MQH_EINVAL, "rule: MQH_RULE_GCV or MQH_RULE_FIXED");
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    if (J < 3 || J > kMaxGrid) return fail(MQH_EINVAL, "n_grid must be 0 or in [3, 4096]");
    if (opts->rule == MQH_RULE_FIXED && (!isfinite(opts->lambda_fixed) || opts->lambda_fixed < 0.0))
        return fail(MQH_EINVAL, "lambda_fixed must be finite and >= 0");
    if (opts->row_scale != 0) return fail(MQH_EINVAL, "the block solve takes row_scale = 0");
    HIPCHK(hipSetDevice(p->device));
    if ((rc = set_row_scale(p, 0))) return rc;
    hipStream_t st = p->stream;
    const uint32_t flags = opts->flags;
    const int64_t n = p->n, ldn = p->ldn;
    const int32_t ell = opts->ell;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const auto t0 = now();
    if (p->mode == MQH_OP_MATFREE_FP32 && nrhs >= 2 && (rc = ensure_multi(p, nrhs, 1))) return rc;
    BlockWs* bw = nullptr;
    if ((rc = block_ws(p, nrhs, ell, &bw))) return rc;
    BlockWs& b = *bw;
    if ((rc = stage_block(p, b, F, ldf, nrhs, flags))) return rc;
    HIPCHK(hipStreamSynchronize(st));
    const auto t1 = now();
    std::vector<double> Ch;
    double E1h[kBlkRhs * kBlkRhs];
    int32_t ld = 0, fl = 0;
    if ((rc = run_gkb_block(p, b, nrhs, ell, Ch, E1h, &ld, &fl, false))) return rc;
    const auto t2 = now();
    if (ld == 0) {
        // nothing to project on: zero coefficients, breakdown reported
        HIPCHK(copy_strided(coef, (size_t)ldc * sizeof(double), b.P, (size_t)ldn * sizeof(double),
                                (size_t)n * sizeof(double), (size_t)nrhs, kind_out(flags), st));
        HIPCHK(hipStreamSynchronize(st));
        if (info)
            for (int32_t k = 0; k < nrhs; ++k) info[k].flags = MQH_INFO_BREAKDOWN;
        return MQH_WBREAKDOWN;
    }
    const int64_t ls = (int64_t)ld * nrhs, ldfull = (int64_t)ell * nrhs;
    double* Y = p->bc->Y;  // ell nrhs x 16, cached with the block workspace
    HIPCHK(hipMemsetAsync(Y, 0, (size_t)ls * kBlkRhs * sizeof(double), st));
    double* svd = sv ? p->bc->sv : nullptr;
    std::vector<ParamOut> po;
    std::vector<int> iters;
    std::vector<char> conv;
    int32_t sweeps = 0;
    bool banded = false;
    if (!(flags & MQH_FLAG_BLOCK_JACOBI) && band_fits((int)ls, nrhs)) {
        if ((rc = band_projected(p, b.Cd, ldfull, b.E1d, nrhs, ld, opts->rule, J, opts->lambda_fixed, Y, svd, po,
                                 &banded)))
            return rc;
        if (banded) {
            iters.assign((size_t)nrhs, 0);
            conv.assign((size_t)nrhs, 1);
        }
    }
    if (!banded && (rc = block_projected(p, b.Cd, ldfull, b.E1d, E1h, nrhs, ld, opts->rule, J, opts->lambda_fixed, Y,
                                         svd, po, iters, conv, &sweeps)))
        return rc;
    const auto t3 = now();
    // coefficients Z Y (in b.P, then out)
    launch_blk_update(b.Z, ldn, n, (int32_t)ls, Y, kBlkRhs, 1, b.P, ldn, nrhs, 0, st);
    LAUNCHCHK("block lift");
    const hipMemcpyKind ko = kind_out(flags);
    HIPCHK(copy_strided(coef, (size_t)ldc * sizeof(double), b.P, (size_t)ldn * sizeof(double),
                            (size_t)n * sizeof(double), (size_t)nrhs, ko, st));
    if (sv) HIPCHK(hipMemcpyAsync(sv, svd, (size_t)ls * sizeof(double), ko, st));
    HIPCHK(hipStreamSynchronize(st));
    const auto t4 = now();
    bool edge = false, noconv = false;
    for (int32_t k = 0; k < nrhs; ++k) {
        edge = edge || (po[(size_t)k].flags & MQH_INFO_GCV_AT_EDGE);
        noconv = noconv || !conv[(size_t)k];
        if (!info) continue;
        mqh_solve_info& I = info[k];
        I.ell_done = ld;
        I.k_chosen = 0;
        I.lambda_chosen = po[(size_t)k].lambda;
        I.crit = po[(size_t)k].crit;
        I.resid_norm = po[(size_t)k].rho;
        I.sol_norm = po[(size_t)k].eta;
        I.flags = po[(size_t)k].flags | (fl ? MQH_INFO_BREAKDOWN : 0u) | (conv[(size_t)k] ? 0u : MQH_INFO_SOLVE_NOCONV) |
                  (banded ? 0u : MQH_INFO_BLOCK_JACOBI);
        I.t_ms[0] = ms(t0, t1);
        I.t_ms[1] = ms(t1, t2);
        I.t_ms[2] = ms(t2, t3);
        I.t_ms[3] = ms(t3, t4);
        I.t_ms[5] = ms(t0, t4);
        I.t_ms[6] = sweeps;
        I.t_ms[7] = iters[(size_t)k];
    }
    if (fl) return MQH_WBREAKDOWN;
    if (noconv) return MQH_WNOCONV;
    if (edge) return MQH_WEDGE;
    return MQH_OK;
}

int mqh_eval(mqh_problem* p, const double* coef, const double* x_eval, int64_t m, double* u, uint32_t flags) {
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (coef == nullptr || x_eval == nullptr || u == nullptr || m < 1) return fail(MQH_EINVAL, "bad eval arguments");
    HIPCHK(hipSetDevice(p->device));
    hipStream_t s = p->stream;
    std::vector<double> xyz((size_t)(3 * m));
    if (flags & MQH_FLAG_DEVICE_PTRS)
        HIPCHK(hipMemcpy(xyz.data(), x_eval, (size_t)(3 * m) * sizeof(double), hipMemcpyDeviceToHost));
    else
        memcpy(xyz.data(), x_eval, (size_t)(3 * m) * sizeof(double));
    if (!all_finite(xyz.data(), 3 * m)) return fail(MQH_EINVAL, "non-finite evaluation point");
    std::vector<double4> rec((size_t)m);
    to_records(p, xyz.data(), m, rec.data(), nullptr);
    const int64_t mb = (m + kBlock - 1) / kBlock;
    int64_t S = (4096 + mb - 1) / mb;
    if (S > 256) S = 256;
    int64_t len = (p->n + S - 1) / S;
    len = round_up(len < 64 ? 64 : len, 2);
    S = (p->n + len - 1) / len;
    const int64_t ldm = round_up(m, 64);
    if (m > p->E_cap) {
        dfree(p->E);
        dfree(p->u);
        p->E_cap = 0;
        if ((rc = dalloc(&p->E, (size_t)m))) return rc;
        if ((rc = dalloc(&p->u, (size_t)ldm))) return rc;
        p->E_cap = m;
    }
    if (S * ldm > p->EP_cap) {
        dfree(p->EP);
        p->EP_cap = 0;
        if ((rc = dalloc(&p->EP, (size_t)(S * ldm)))) return rc;
        p->EP_cap = S * ldm;
    }
    if ((rc = stage_in(p->vx, coef, p->n, flags, s))) return rc;
    HIPCHK(hipMemcpyAsync(p->E, rec.data(), (size_t)m * sizeof(double4), hipMemcpyHostToDevice, s));
    launch_eval_partial(p->X64, p->vx, p->n, p->E, m, (int)S, len, p->ec, p->EP, ldm, s);
    LAUNCHCHK("evaluation");
    launch_reduce_slices(p->EP, ldm, (int)S, m, nullptr, nullptr, 0.0, nullptr, p->u, nullptr, s);
    LAUNCHCHK("evaluation reduction");
    HIPCHK(hipMemcpyAsync(u, p->u, (size_t)m * sizeof(double), kind_out(flags), s));
    HIPCHK(hipStreamSynchronize(s));
    return MQH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Standalone projected-problem calls (own temporary buffers)
// ---------------------------------------------------------------------------

namespace {
struct Tmp {
    std::vector<void*> bufs;
    ~Tmp() {
        for (void* b : bufs) dfree_raw(b);
    }
    template <typename T>
    int get(T** p, size_t count) {
        int rc = dalloc(p, count);
        if (rc == MQH_OK) bufs.push_back((void*)*p);
        return rc;
    }
};

// device copy of an input array (returns the device pointer to use)
template <typename T>
int dev_in(Tmp& t, const T* src, size_t count, uint32_t flags, hipStream_t s, const T** out) {
    if (flags & MQH_FLAG_DEVICE_PTRS) {
        *out = src;
        return MQH_OK;
    }
    T* d;
    int rc = t.get(&d, count);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, s));
    *out = d;
    return MQH_OK;
}

template <typename T>
int dev_out(Tmp& t, T* dst, size_t count, uint32_t flags, T** out) {
    if (flags & MQH_FLAG_DEVICE_PTRS) {
        *out = dst;
        return MQH_OK;
    }
    return t.get(out, count);
}
}  // namespace

extern "C" {

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free projected SVD: the workspace of the projected SVD (left
// vectors, Gram matrix, bidiagonal and bookkeeping; the QR fallback's
// rotation matrix), the status word, and V when the caller does not want it, lives
// in one file-scope device array.  Host code never passes the array's name
// to a kernel or a copy: its device address is looked up once per device
// (hipGetSymbolAddress) and kept in g_scratch_addr.
// ---------------------------------------------------------------------------

constexpr int kNoAllocMaxEll = MQH_NOALLOC_MAX_ELL;
constexpr size_t kScratchWs = svd_ws_doubles(kNoAllocMaxEll);             // the projected SVD's workspace
constexpr size_t kScratchMat = (size_t)kNoAllocMaxEll * kNoAllocMaxEll;  // V when the caller passes none
constexpr size_t kScratchDoubles = kScratchWs + kScratchMat + 32;         // + status (and padding)
static_assert(MQH_NOALLOC_SCRATCH_BYTES == kScratchDoubles * sizeof(double), "scratch size in the header");

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on
// the first call on that device).
int scratch_addr(double** out) {
    *out = nullptr;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MQH_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr) return fail(MQH_EDEVICE, "scratch array has no device address");
        g_scratch_addr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[dev];
    return MQH_OK;
}
}  // namespace

extern "C" {

int mqh_proj_svd_noalloc(const double* alpha, const double* beta, int32_t ell, double* sv, double* ftil, double* V,
                         void* stream) {
    if (alpha == nullptr || beta == nullptr || sv == nullptr || ftil == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (ell < 1 || ell > kNoAllocMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= MQH_NOALLOC_MAX_ELL");
    hipStream_t s = (hipStream_t)stream;
    double* base = nullptr;
    int rc;
    if ((rc = scratch_addr(&base))) return rc;
    double* dws = base;
    double* dV = V != nullptr ? V : base + kScratchWs;
    int32_t* dst = reinterpret_cast<int32_t*>(base + kScratchWs + kScratchMat);
    // the kernels write every workspace entry and the status word before
    // reading them; nothing in the scratch array has to start at zero
    launch_bidiag_svd(alpha, beta, ell, nullptr, dws, sv, ftil, dV, ell, dst, 0, s);
    LAUNCHCHK("projected SVD");
    int32_t status = 0;
    HIPCHK(hipMemcpyAsync(&status, dst, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (status < 0) return fail(MQH_EDEVICE, "projected SVD did not converge");
    return MQH_OK;
}

int mqh_proj_svd(const double* alpha, const double* beta, int32_t ell, double* sv, double* ftil, double* V,
                 void* stream, uint32_t flags) {
    if (alpha == nullptr || beta == nullptr || sv == nullptr || ftil == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (ell < 1 || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= MQH_MAX_ELL");
    if ((flags & MQH_FLAG_PROJ_QR) && (flags & MQH_FLAG_PROJ_NO_FALLBACK))
        return fail(MQH_EINVAL, "MQH_FLAG_PROJ_QR and MQH_FLAG_PROJ_NO_FALLBACK exclude each other");
    if (!(flags & MQH_FLAG_DEVICE_PTRS) && (!all_finite(alpha, ell) || !all_finite(beta, ell + 1)))
        return fail(MQH_EINVAL, "non-finite input");
    const int mode = (flags & MQH_FLAG_PROJ_QR) ? 1 : (flags & MQH_FLAG_PROJ_NO_FALLBACK) ? 2 : 0;
    hipStream_t s = (hipStream_t)stream;
    Tmp t;
    int rc;
    const double *da, *db;
    double *dsv, *dft, *dV, *dws;
    int32_t* dst;
    if ((rc = dev_in(t, alpha, (size_t)ell, flags, s, &da))) return rc;
    if ((rc = dev_in(t, beta, (size_t)ell + 1, flags, s, &db))) return rc;
    if ((rc = dev_out(t, sv, (size_t)ell, flags, &dsv))) return rc;
    if ((rc = dev_out(t, ftil, (size_t)ell + 1, flags, &dft))) return rc;
    if (V != nullptr) {
        if ((rc = dev_out(t, V, (size_t)ell * ell, flags, &dV))) return rc;
    } else if ((rc = t.get(&dV, (size_t)ell * ell))) {
        return rc;
    }
    if ((rc = t.get(&dws, svd_ws_doubles(ell)))) return rc;
    if ((rc = t.get(&dst, 1))) return rc;
    launch_bidiag_svd(da, db, ell, nullptr, dws, dsv, dft, dV, ell, dst, mode, s);
    LAUNCHCHK("projected SVD");
    int32_t status = 0;
    HIPCHK(hipMemcpyAsync(&status, dst, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) {
        HIPCHK(hipMemcpyAsync(sv, dsv, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ftil, dft, (size_t)(ell + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        if (V) HIPCHK(hipMemcpyAsync(V, dV, (size_t)ell * ell * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (status < 0) return fail(MQH_EDEVICE, "projected SVD did not converge");
    if (status == 2) return fail(MQH_EDEVICE, "projected SVD: the fast path failed its acceptance test");
    return MQH_OK;
}

int mqh_param_choice(const double* sv, const double* ftil, int32_t ell, int32_t method, int32_t rule, int32_t n_grid,
                     double lambda_fixed, int32_t k_trunc, double gcv_weight, double* lambda, int32_t* k, double* crit,
                     uint32_t* info_flags, double* curve, void* stream, uint32_t flags) {
    if (sv == nullptr || ftil == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (ell < 1 || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= MQH_MAX_ELL");
    if (method != MQH_METHOD_INE_TSVD && method != MQH_METHOD_HKT) return fail(MQH_EINVAL, "method");
    if (rule < MQH_RULE_GCV || rule > MQH_RULE_WGCV) return fail(MQH_EINVAL, "rule");
    if (rule == MQH_RULE_WGCV && !(gcv_weight > 0.0 && gcv_weight <= 1.0))
        return fail(MQH_EINVAL, "gcv_weight must be in (0, 1]");
    const int32_t J = n_grid == 0 ? 200 : n_grid;
    if (J < 3 || J > kMaxGrid) return fail(MQH_EINVAL, "n_grid must be 0 or in [3, 4096]");
    if (method == MQH_METHOD_HKT && rule == MQH_RULE_FIXED && (!isfinite(lambda_fixed) || lambda_fixed < 0.0))
        return fail(MQH_EINVAL, "lambda_fixed");
    if (method == MQH_METHOD_INE_TSVD && rule == MQH_RULE_FIXED && (k_trunc < 1 || k_trunc > ell))
        return fail(MQH_EINVAL, "k_trunc");
    if (!(flags & MQH_FLAG_DEVICE_PTRS) && (!all_finite(sv, ell) || !all_finite(ftil, ell + 1)))
        return fail(MQH_EINVAL, "non-finite input");
    hipStream_t s = (hipStream_t)stream;
    Tmp t;
    int rc;
    const double *dsv, *dft;
    double* dcurve = nullptr;
    ParamOut* dpo;
    if ((rc = dev_in(t, sv, (size_t)ell, flags, s, &dsv))) return rc;
    if ((rc = dev_in(t, ftil, (size_t)ell + 1, flags, s, &dft))) return rc;
    if (curve != nullptr && (rc = dev_out(t, curve, (size_t)J, flags, &dcurve))) return rc;
    if ((rc = t.get(&dpo, 1))) return rc;
    launch_param_choice(dsv, dft, ell, nullptr, method, rule, J, lambda_fixed, k_trunc, gcv_weight, dcurve, dpo, s);
    LAUNCHCHK("parameter choice");
    ParamOut po;
    HIPCHK(hipMemcpyAsync(&po, dpo, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    if (curve != nullptr && !(flags & MQH_FLAG_DEVICE_PTRS))
        HIPCHK(hipMemcpyAsync(curve, dcurve, (size_t)J * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (lambda) *lambda = po.lambda;
    if (k) *k = po.k;
    if (crit) *crit = po.crit;
    if (info_flags) *info_flags = po.flags;
    return (po.flags & (MQH_INFO_GCV_AT_EDGE | MQH_INFO_LCURVE_AT_EDGE)) ? MQH_WEDGE : MQH_OK;
}

int mqh_lsqr(const double* alpha, const double* beta, int32_t ell, int64_t n, int32_t rule, int32_t k_trunc, int32_t* k,
             double* crit, uint32_t* info_flags, double* y, double* rho, double* eta, void* stream, uint32_t flags) {
    if (alpha == nullptr || beta == nullptr || y == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (ell < 1 || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= MQH_MAX_ELL");
    if (n < ell) return fail(MQH_EINVAL, "need n >= ell");
    if (rule < MQH_RULE_GCV || rule > MQH_RULE_FIXED) return fail(MQH_EINVAL, "rule");
    if (rule == MQH_RULE_FIXED && (k_trunc < 1 || k_trunc > ell)) return fail(MQH_EINVAL, "k_trunc");
    if (!(flags & MQH_FLAG_DEVICE_PTRS) && (!all_finite(alpha, ell) || !all_finite(beta, ell + 1)))
        return fail(MQH_EINVAL, "non-finite input");
    hipStream_t s = (hipStream_t)stream;
    Tmp t;
    int rc;
    const double *da, *db;
    double *dy, *drho = nullptr, *deta = nullptr;
    ParamOut* dpo;
    if ((rc = dev_in(t, alpha, (size_t)ell, flags, s, &da))) return rc;
    if ((rc = dev_in(t, beta, (size_t)ell + 1, flags, s, &db))) return rc;
    if ((rc = dev_out(t, y, (size_t)ell, flags, &dy))) return rc;
    if (rho != nullptr && (rc = dev_out(t, rho, (size_t)ell, flags, &drho))) return rc;
    if (eta != nullptr && (rc = dev_out(t, eta, (size_t)ell, flags, &deta))) return rc;
    if ((rc = t.get(&dpo, 1))) return rc;
    launch_lsqr(da, db, ell, nullptr, n, rule, k_trunc, drho, deta, dpo, dy, ell, s);
    LAUNCHCHK("LSQR iterates");
    ParamOut po;
    HIPCHK(hipMemcpyAsync(&po, dpo, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) {
        HIPCHK(hipMemcpyAsync(y, dy, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
        if (rho) HIPCHK(hipMemcpyAsync(rho, drho, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
        if (eta) HIPCHK(hipMemcpyAsync(eta, deta, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (k) *k = po.k;
    if (crit) *crit = po.crit;
    if (info_flags) *info_flags = po.flags;
    return (po.flags & MQH_INFO_LCURVE_AT_EDGE) ? MQH_WEDGE : MQH_OK;
}

int mqh_proj_solution(const double* sv, const double* ftil, const double* V, int32_t ell, int32_t method, double lambda,
                      int32_t k, double* y, void* stream, uint32_t flags) {
    if (sv == nullptr || ftil == nullptr || V == nullptr || y == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (ell < 1 || ell > kMaxEll) return fail(MQH_EINVAL, "need 1 <= ell <= MQH_MAX_ELL");
    if (method != MQH_METHOD_INE_TSVD && method != MQH_METHOD_HKT) return fail(MQH_EINVAL, "method");
    if (method == MQH_METHOD_HKT && (!isfinite(lambda) || lambda < 0.0)) return fail(MQH_EINVAL, "lambda");
    if (method == MQH_METHOD_INE_TSVD && (k < 1 || k > ell)) return fail(MQH_EINVAL, "k");
    hipStream_t s = (hipStream_t)stream;
    Tmp t;
    int rc;
    const double *dsv, *dft, *dV;
    double* dy;
    if ((rc = dev_in(t, sv, (size_t)ell, flags, s, &dsv))) return rc;
    if ((rc = dev_in(t, ftil, (size_t)ell + 1, flags, s, &dft))) return rc;
    if ((rc = dev_in(t, V, (size_t)ell * ell, flags, s, &dV))) return rc;
    if ((rc = dev_out(t, y, (size_t)ell, flags, &dy))) return rc;
    launch_proj_solution(dsv, dft, dV, ell, ell, nullptr, method, lambda, k, nullptr, dy, ell, s);
    LAUNCHCHK("projected solution");
    if (!(flags & MQH_FLAG_DEVICE_PTRS))
        HIPCHK(hipMemcpyAsync(y, dy, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MQH_OK;
}

int mqh_lift(const double* Z, int64_t n, int32_t ell, const double* y, double* coef, void* stream, uint32_t flags) {
    if (Z == nullptr || y == nullptr || coef == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (n < 1 || ell < 1) return fail(MQH_EINVAL, "need n >= 1, ell >= 1");
    hipStream_t s = (hipStream_t)stream;
    Tmp t;
    int rc;
    const double *dZ, *dy;
    double* dc;
    if ((rc = dev_in(t, Z, (size_t)(n * ell), flags, s, &dZ))) return rc;
    if ((rc = dev_in(t, y, (size_t)ell, flags, s, &dy))) return rc;
    if ((rc = dev_out(t, coef, (size_t)n, flags, &dc))) return rc;
    launch_lift(dZ, n, n, ell, nullptr, dy, dc, s);
    LAUNCHCHK("lift");
    if (!(flags & MQH_FLAG_DEVICE_PTRS))
        HIPCHK(hipMemcpyAsync(coef, dc, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MQH_OK;
}


// ---------------------------------------------------------------------------
// Predictor network (device pointers only) and the learned solve
// ---------------------------------------------------------------------------

int mqh_mlp_forward(const float* params, const float* x, int32_t batch, float* y, float* hidden, void* stream,
                    uint32_t flags) {
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) return fail(MQH_EINVAL, "the network calls take device pointers only");
    if (params == nullptr || x == nullptr || y == nullptr || hidden == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (batch < 1) return fail(MQH_EINVAL, "batch must be >= 1");
    launch_mlp_forward(params, x, batch, y, hidden, (hipStream_t)stream);
    LAUNCHCHK("network forward");
    return MQH_OK;
}

int mqh_mlp_backward(const float* params, const float* x, const float* hidden, const float* dy, int32_t batch,
                     float* grad, float* work, void* stream, uint32_t flags) {
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) return fail(MQH_EINVAL, "the network calls take device pointers only");
    if (params == nullptr || x == nullptr || hidden == nullptr || dy == nullptr || grad == nullptr || work == nullptr)
        return fail(MQH_EINVAL, "NULL array");
    if (batch < 1) return fail(MQH_EINVAL, "batch must be >= 1");
    launch_mlp_backward(params, x, hidden, dy, batch, grad, work, (hipStream_t)stream);
    LAUNCHCHK("network backward");
    return MQH_OK;
}

int mqh_mlp_loss(const float* y, const float* t, const float* w, int32_t batch, float* loss, float* dy, void* stream,
                 uint32_t flags) {
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) return fail(MQH_EINVAL, "the network calls take device pointers only");
    if (y == nullptr || t == nullptr || w == nullptr || (loss == nullptr && dy == nullptr))
        return fail(MQH_EINVAL, "NULL array");
    if (batch < 1) return fail(MQH_EINVAL, "batch must be >= 1");
    launch_mse(y, t, w, batch, loss, dy, (hipStream_t)stream);
    LAUNCHCHK("network loss");
    return MQH_OK;
}

int mqh_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, void* stream, uint32_t flags) {
    if (!(flags & MQH_FLAG_DEVICE_PTRS)) return fail(MQH_EINVAL, "the network calls take device pointers only");
    if (params == nullptr || grad == nullptr || m == nullptr || v == nullptr) return fail(MQH_EINVAL, "NULL array");
    if (n < 1 || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(MQH_EINVAL, "bad Adam arguments");
    launch_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    LAUNCHCHK("Adam step");
    return MQH_OK;
}

int mqh_solve_learned(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts,
                      const mqh_predictor* pred, double* coef, mqh_solve_info* info, mqh_learned_info* linfo) {
    clear_info(info);
    if (linfo) memset(linfo, 0, sizeof(*linfo));
    int rc;
    if ((rc = check_problem(p))) return rc;
    if (opts == nullptr || pred == nullptr || pred->params == nullptr) return fail(MQH_EINVAL, "NULL opts / predictor");
    if (coef == nullptr) return fail(MQH_EINVAL, "NULL coef");
    if ((p->n_int > 0 && f_int == nullptr) || (p->n_bnd > 0 && g_bnd == nullptr)) return fail(MQH_EINVAL, "NULL data");
    const int32_t ell = opts->ell;
    if (ell < kMlpProbe || ell > p->n || ell > kMaxEll)
        return fail(MQH_EINVAL, "need MQH_MLP_PROBE <= ell <= min(n, MQH_MAX_ELL)");
    if (opts->reorth != 0 && opts->reorth != 1) return fail(MQH_EINVAL, "reorth must be 0 or 1");
    if (opts->method != MQH_METHOD_HKT || opts->rule != MQH_RULE_GCV)
        return fail(MQH_EINVAL, "the learned solve is HKT with GCV as judge and fallback");
    if (opts->row_scale != 0 && opts->row_scale != 1) return fail(MQH_EINVAL, "row_scale must be 0 or 1");
    const int32_t J = opts->n_grid == 0 ? 200 : opts->n_grid;
    if (J < 3 || J > kMaxGrid) return fail(MQH_EINVAL, "n_grid must be 0 or in [3, 4096]");
    if (!(pred->h > 0.0) || !isfinite(pred->h) || pred->ell_step < 1 ||
        !(pred->judge_ratio == 0.0 || pred->judge_ratio >= 1.0))
        return fail(MQH_EINVAL, "predictor needs h > 0, ell_step >= 1, judge_ratio 0 or >= 1");
    if (!(p->kappa > 0.0)) return fail(MQH_EINVAL, "the predictor's features need kappa > 0");
    for (int i = 0; i < kMlpIn; ++i)
        if (!(pred->in_std[i] > 0.0f) || !isfinite(pred->in_mean[i])) return fail(MQH_EINVAL, "bad standardisation");
    for (int i = 0; i < kMlpOut; ++i)
        if (!(pred->out_std[i] > 0.0f) || !isfinite(pred->out_mean[i])) return fail(MQH_EINVAL, "bad standardisation");
    const uint32_t flags = opts->flags;
    HIPCHK(hipSetDevice(p->device));
    // with the row scaling the whole run is on D A and D f: the features come
    // from its scalars, so the predictor must have been trained on such runs
    if ((rc = set_row_scale(p, opts->row_scale))) return rc;
    hipStream_t s = p->stream;
    if ((rc = ensure_gkb(p, ell))) return rc;
    const size_t mlp_floats = kMlpIn + kMlpOut + 3 * kMlpWidth + 2 * kMlpIn;
    if (p->mlp == nullptr && (rc = dalloc(&p->mlp, mlp_floats))) return rc;
    if (p->pout2 == nullptr && (rc = dalloc(&p->pout2, 1))) return rc;
    float* dx = p->mlp;
    float* dyv = dx + kMlpIn;
    float* dhid = dyv + kMlpOut;
    float* dmean = dhid + 3 * kMlpWidth;
    float* dstd = dmean + kMlpIn;
    for (auto& e : p->pev) (void)hipEventDestroy(e);
    p->pev.clear();
    HIPCHK(hipEventRecord(p->ev[0], s));
    HIPCHK(hipMemcpyAsync(dmean, pred->in_mean, kMlpIn * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dstd, pred->in_std, kMlpIn * sizeof(float), hipMemcpyHostToDevice, s));
    if ((rc = stage_in(p->vx, f_int, p->n_int, flags, s))) return rc;
    if ((rc = stage_in(p->vx + p->n_int, g_bnd, p->n_bnd, flags, s))) return rc;
    if ((rc = scale_rhs(p, p->vx, 1, 0))) return rc;
    HIPCHK(hipEventRecord(p->ev[1], s));
    // probe: the first kMlpProbe steps, then the network
    if ((rc = run_gkb(p, ell, opts->reorth, false, 0, kMlpProbe))) return rc;
    launch_mlp_features(p->alpha, p->beta, p->kappa, p->eps, (double)p->n, pred->h, dmean, dstd, dx, s);
    launch_mlp_forward(pred->params, dx, 1, dyv, dhid, s);
    LAUNCHCHK("predictor");
    float yo[kMlpOut];
    double a1 = 0.0;
    HIPCHK(hipMemcpyAsync(yo, dyv, sizeof(yo), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&a1, p->alpha, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&p->hres->st, p->st, sizeof(GkbState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double t0 = (double)yo[0] * pred->out_std[0] + pred->out_mean[0];
    const double t1 = (double)yo[1] * pred->out_std[1] + pred->out_mean[1];
    int32_t ell_pred = ell;
    if (isfinite(t1)) {
        const double want = t1 * (double)ell;
        const double q = ceil(want / (double)pred->ell_step) * (double)pred->ell_step;
        ell_pred = q < (double)kMlpProbe ? kMlpProbe : (q > (double)ell ? ell : (int32_t)q);
    }
    if (p->hres->st.stopped) ell_pred = p->hres->st.ell_done > kMlpProbe ? kMlpProbe : p->hres->st.ell_done;
    const double lam_net = isfinite(t0) && a1 > 0.0 ? a1 * exp(t0) : 0.0;
    // the rest of the run, then the projected problem with GCV as judge
    if ((rc = run_gkb(p, ell, opts->reorth, false, kMlpProbe, ell_pred))) return rc;
    launch_cap_ell(p->st, ell_pred, s);
    HIPCHK(hipEventRecord(p->ev[2], s));
    const int32_t* lp = &p->st->ell_done;
    launch_fill(p->sv, ell, 0.0, s);
    launch_bidiag_svd(p->alpha, p->beta, ell, lp, p->Vw, p->sv, p->ftil, p->V, ell, p->svd_status, 0, s);
    LAUNCHCHK("projected SVD");
    HIPCHK(hipEventRecord(p->ev[3], s));
    launch_param_choice(p->sv, p->ftil, ell, lp, MQH_METHOD_HKT, MQH_RULE_GCV, J, 0.0, 0, 1.0, nullptr, p->pout, s);
    launch_param_choice(p->sv, p->ftil, ell, lp, MQH_METHOD_HKT, MQH_RULE_FIXED, J, lam_net, 0, 1.0, nullptr, p->pout2,
                        s);
    LAUNCHCHK("parameter choice");
    ParamOut po_gcv, po_net;
    std::vector<double> svh((size_t)ell);
    HIPCHK(hipMemcpyAsync(&po_gcv, p->pout, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&po_net, p->pout2, sizeof(ParamOut), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&p->hres->svd_status, p->svd_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&p->hres->st, p->st, sizeof(GkbState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(svh.data(), p->sv, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (p->hres->svd_status < 0) return fail(MQH_EDEVICE, "projected SVD did not converge");
    // GCV's search range at ell_pred: a network lambda more than 10x outside it is an extrapolation
    const int32_t le = p->hres->st.ell_done;
    bool use_net = lam_net > 0.0 && isfinite(lam_net) && le >= 1;
    if (use_net) {
        const double hi = svh[0];
        const double lo = svh[le - 1] > 16.0 * DBL_EPSILON * hi ? svh[le - 1] : 16.0 * DBL_EPSILON * hi;
        use_net = lam_net >= 0.1 * lo && lam_net <= 10.0 * hi;
    }
    if (use_net && pred->judge_ratio >= 1.0) use_net = isfinite(po_net.crit) && po_net.crit <= pred->judge_ratio * po_gcv.crit;
    const ParamOut& po = use_net ? po_net : po_gcv;
    launch_proj_solution(p->sv, p->ftil, p->V, ell, ell, lp, MQH_METHOD_HKT, po.lambda, 0, nullptr, p->y, ell, s);
    HIPCHK(hipEventRecord(p->ev[4], s));
    launch_lift(p->Z, p->ldn, p->n, ell, lp, p->y, p->coef, s);
    LAUNCHCHK("lift");
    HIPCHK(hipEventRecord(p->ev[5], s));
    HIPCHK(hipMemcpyAsync(&p->hres->st, p->st, sizeof(GkbState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(coef, p->coef, (size_t)p->n * sizeof(double), kind_out(flags), s));
    HIPCHK(hipEventRecord(p->ev[6], s));
    HIPCHK(hipStreamSynchronize(s));
    const GkbState& st = p->hres->st;
    uint32_t iflags = use_net ? 0u : po_gcv.flags;
    if (st.flag != 0) iflags |= MQH_INFO_BREAKDOWN;
    if (p->hres->svd_status == 1) iflags |= MQH_INFO_SVD_QR;
    if (info) {
        info->ell_done = st.ell_done;
        info->k_chosen = 0;
        info->lambda_chosen = po.lambda;
        info->crit = po.crit;
        info->resid_norm = po.rho;
        info->sol_norm = po.eta;
        info->flags = iflags;
        float ms = 0.f;
        const int pairs[6][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {0, 6}};
        for (int q = 0; q < 6; ++q)
            if (hipEventElapsedTime(&ms, p->ev[pairs[q][0]], p->ev[pairs[q][1]]) == hipSuccess) info->t_ms[q] = ms;
    }
    if (linfo) {
        linfo->ell_pred = ell_pred;
        linfo->used_net_lambda = use_net ? 1 : 0;
        linfo->lambda_net = lam_net;
        linfo->lambda_gcv = po_gcv.lambda;
        linfo->gcv_net = po_net.crit;
        linfo->gcv_min = po_gcv.crit;
        linfo->out[0] = t0;
        linfo->out[1] = t1;
    }
    if (st.flag != 0) return MQH_WBREAKDOWN;
    if (iflags & MQH_INFO_GCV_AT_EDGE) return MQH_WEDGE;
    return MQH_OK;
}

}  // extern "C"
