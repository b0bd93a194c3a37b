// Host runtime and C-ABI of libfdtdb: grid layout, material tables, validation,
// region partition, launch sequencing, HIP graph capture and read-out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdtdb.h"
#include "fdtdb_internal.h"

namespace fdtdb {
hipError_t launch_update_e(int dim, bool f64, const EArgs &a, const double *coef_host, int kind, int ng, bool pml,
                           bool energy, hipStream_t s);
hipError_t launch_update_h(int dim, bool f64, const HArgs &a, bool pml, hipStream_t s);
hipError_t launch_tick(Clock *clk, const SourceDev *src, int nsrc, double dt, hipStream_t s);
hipError_t launch_energy_reduce(const Clock *clk, const double *partial, long long nslots, int every, double *out,
                                long long capacity, hipStream_t s);

hipError_t launch_dft_stage(bool f64, const DftArgs &a, hipStream_t s);
hipError_t launch_dft_flush(const Clock *clk, const double *omega, int nf, int nslots, double dt, double *tw,
                            const double *stage, int npts, double2 *acc, hipStream_t s);
hipError_t launch_dft_flux(const double2 *acc, const double2 *acc_im, int npts, int nf, double *flux, hipStream_t s);
hipError_t launch_nonfinite(bool f64, const void *f, long long n, int *flag, hipStream_t s);
hipError_t launch_to_f64(bool f64, const void *src, long long n, double *dst, hipStream_t s);
hipError_t launch_bath16_to_f64(const void *src, long long n, int yf, double inv_s, double *dst, hipStream_t s);
hipError_t launch_probe(bool f64, const void *E, const void *P, const int *q, const int *m, int n, const Clock *clk,
                        long long capacity, float *outE, float *outP, hipStream_t s);
}  // namespace fdtdb

using namespace fdtdb;

namespace {

thread_local std::string g_err;

fdtdb_status fail(fdtdb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(x)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(FDTDB_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define TRY(x)                          \
    do {                                \
        fdtdb_status s_ = (x);          \
        if (s_ != FDTDB_OK) return s_;  \
    } while (0)

uint64_t fnv1a(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    uint64_t h = 1469598103934665603ULL;
    for (size_t i = 0; i < n; i++) { h ^= c[i]; h *= 1099511628211ULL; }
    return h;
}

struct Material {
    int kind = K_BACKGROUND;
    int64_t lo[3], hi[3];
    int mext[3];
    long long mcells = 0;
    double eps = 1.0, omega0 = 0.0, gamma0 = 0.0, sigma0 = 0.0, sigma_max = 0.0;
    bool sigma_per_cell = false;
    int nb = 0, ng = 0;
    int nterm = 0;                   // multi-term material: Lorentz / Drude terms
    std::vector<double> wj, gj, kj, coef;
    void *P[2][3] = {};
    void *Y[2][3] = {};
    void *sigma_dev = nullptr;
    double *coef_dev = nullptr;
    // learned closure
    float *cw_dev = nullptr;
    void *hid[3] = {};
    double cscale[4] = {1.0, 1.0, 1.0, 1.0};
    // FNV-1a of the per-cell sigma values and of the closure weights as given (checkpoint fingerprint)
    uint64_t sigma_hash = 0, weight_hash = 0;
    // bath coordinate storage: 0 the state type, 1 binary16 or 2 bfloat16 of Y * yscale
    int yfmt = 0;
    double yscale = 1.0;
    // thermal bath (kT > 0, noise key from seed) and anharmonic bath (lam, one per mode)
    double kT = 0.0;
    uint64_t seed = 0;
    std::vector<double> lam;
    int bext() const { return (kT > 0.0 ? 1 : 0) | (lam.empty() ? 0 : 2); }
};

struct Region {
    int lo[3], hi[3];
    int mat = -1;
    int pml_mask = 0;
    double eps = 1.0;
    void *psiE[3][2] = {};
    void *psiH[3][2] = {};
    bool energy = false;
    // on a Bloch pair: the region reads the other part (E: the first row along a Bloch axis, whose lower
    // neighbour wraps; H: the last row, whose upper neighbour wraps) and takes the generic kernels; a 2D
    // Lorentz-Bath material touching the wrap is one such region as a whole, on its load-first kernel
    bool wrap = false;
    long long block_base = 0;
    // H only: z-term psi for z < zlo and z >= zhi alone, in zw = (zlo - lo) + (hi - zhi) slots per
    // row; zw = 0: per cell of the region
    int zlo = 0, zhi = 0, zw = 0;
    long long cells() const { return (long long)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
    long long psi_words(int axis) const { return zw && axis == 2 ? cells() / (hi[2] - lo[2]) * zw : cells(); }
};

// one kernel launch of a step: a single region, or a group of background regions (grouped
// launches replace many small launches whose cost is mostly launch latency)
struct Launch {
    std::vector<int> regs;
    bool grouped = false, v4 = false, pml = false, energy = false;
    long long blocks = 0, cells = 0, block_base = 0;
    RegionTable *rd = nullptr;
};

struct Pending {
    int rec;
    hipEvent_t a, b;
};

struct Source {
    int comp;
    int64_t lo[3], hi[3];
    double omega_c, width, amplitude, eps;
    std::vector<double> profile;
    double *profile_dev = nullptr;
};

struct Dft {
    int axis;
    int64_t lo[3], hi[3];
    int npts, nf;
    int t1, t2;
    std::vector<double> omega;
    double *omega_dev = nullptr, *stage = nullptr, *tw = nullptr, *flux_dev = nullptr;
    double2 *acc = nullptr;
    int nstaged = 0;
};

struct Energy {
    int64_t lo[3], hi[3];
    int every;
    double *partial = nullptr;
    long long nslots = 0;
    double *out = nullptr;
    long long capacity = 0;
    // watchdog over a monitor that spans the whole grid: samples examined so far, the first total
    // after every source has ended, and the smallest total since
    long long checked = 0;
    double ref = -1.0, low = 0.0;
};

// trajectory recorder: E^{n+1/2} and the new P^{n+3/2} at chosen cells of one material, steps
// [0, capacity)
struct Probe {
    int mat, comp, n;
    long long capacity;
    int *q = nullptr, *m = nullptr;      // grid and material-box indices of the cells
    float *E = nullptr, *P = nullptr;    // [capacity][n]
};

size_t words(long long n, bool f64) { return (size_t)n * (f64 ? 8 : 4); }

}  // namespace

struct fdtdb_grid_s {
    int ndim = 3;
    int n[3] = {1, 1, 1};
    long long ncell = 0;
    double dt = 0.5, R0 = 1e-8;
    bool f64 = false;
    int bc[3], pml[3];
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *E[3] = {}, *H[3] = {};
    std::vector<Material> mats;
    std::vector<Source> srcs;
    std::vector<Dft> dfts;
    std::vector<Energy> ens;
    std::vector<Probe> probes;
    std::vector<Region> regions;    // E / material update regions
    std::vector<Region> hregions;   // H update regions (CPML partition only)
    std::vector<Launch> elaunch, hlaunch;
    double *pml_b[3] = {}, *pml_c[3] = {}, *pml_bh[3] = {}, *pml_ch[3] = {};
    Clock *clock = nullptr;
    SourceDev *src_dev = nullptr;
    int *flag_dev = nullptr;
    bool finalized = false;
    long long steps = 0;          // steps enqueued
    // Bloch pair: the grid of the other part, this grid's part (0 real, 1 imaginary), the phase of each
    // axis; orphan: the other part was destroyed (this grid can no longer step)
    fdtdb_grid_s *twin = nullptr;
    int part = 0;
    double bph[3] = {0.0, 0.0, 0.0};
    bool orphan = false;
    long long total_blocks = 0;   // E-kernel blocks over all regions (energy partial slots)
    // graphs
    int graph_chunk = 0;
    hipGraphExec_t graph = nullptr;
    int graph_parity = 0;
    int launches_per_step = 0;
    std::vector<void *> allocs;
    std::map<void *, size_t> sizes;   // bytes of every live allocation (checkpoint layout)
    // profiling
    int profiling = 0;             // 0 off, 1 every E/H launch, 2 dispersive-material E launches only
    std::vector<fdtdb_kernel_record> records;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    std::map<void *, void *> bases;   // allocations handed out at an offset: their start
    DevAllocator mem = current_allocator();
    // bytes of device memory, zeroed; offset > 0 (a multiple of 256) hands out the memory that many
    // bytes past the start of the allocation
    fdtdb_status alloc(void **p, size_t bytes, size_t offset = 0) {
        if (bytes == 0) bytes = 8;
        void *b = nullptr;
        hipError_t e = dev_alloc(mem, &b, bytes + offset);
        if (e != hipSuccess) return fail(FDTDB_E_NOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
        // the zeroing runs on the null stream, asynchronously to the host; the grid's own stream is
        // non-blocking, so wait for it here: otherwise a kernel enqueued next on that stream (a
        // read-out's conversion into a fresh buffer) could run first and then be overwritten
        e = hipMemset(b, 0, bytes + offset);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return fail(FDTDB_E_DEVICE, "hipMemset: %s", hipGetErrorString(e));
        allocs.push_back(b);
        *p = static_cast<char *>(b) + offset;
        if (offset) bases[*p] = b;
        sizes[*p] = bytes;
        return FDTDB_OK;
    }
    void release(void *&p) {
        if (!p) return;
        sizes.erase(p);
        auto it = bases.find(p);
        void *b = it == bases.end() ? p : it->second;
        if (it != bases.end()) bases.erase(it);
        for (auto &q : allocs)
            if (q == b) {
                dev_free(mem, q);
                q = allocs.back();
                allocs.pop_back();
                break;
            }
        p = nullptr;
    }
    size_t esize() const { return f64 ? 8 : 4; }
};

namespace {

bool box_ok(const fdtdb_grid_s *g, const fdtdb_box *b) {
    if (!b) return false;
    for (int a = 0; a < 3; a++)
        if (b->lo[a] < 0 || b->hi[a] > g->n[a] || b->lo[a] >= b->hi[a]) return false;
    return true;
}

bool overlap(const int64_t *alo, const int64_t *ahi, const int64_t *blo, const int64_t *bhi) {
    for (int a = 0; a < 3; a++)
        if (ahi[a] <= blo[a] || bhi[a] <= alo[a]) return false;
    return true;
}

bool in_pml(const fdtdb_grid_s *g, const int64_t *lo, const int64_t *hi) {
    for (int a = 0; a < 3; a++) {
        if (g->bc[a] != FDTDB_BC_PML) continue;
        if (lo[a] < g->pml[a] || hi[a] > g->n[a] - g->pml[a]) return true;
    }
    return false;
}

fdtdb_status check_new_material(fdtdb_grid_s *g, const fdtdb_box *box, bool dispersive) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "materials must be set before the first step");
    if (!box_ok(g, box)) return fail(FDTDB_E_INVALID, "material box outside the grid or empty");
    for (auto &m : g->mats)
        if (overlap(box->lo, box->hi, m.lo, m.hi)) return fail(FDTDB_E_INVALID, "material boxes overlap");
    if (in_pml(g, box->lo, box->hi))
        return fail(FDTDB_E_INVALID, dispersive ? "dispersive material inside the CPML layer"
                                                : "material inside the CPML layer (the layer assumes eps_inf = 1)");
    if (g->mats.size() >= 4096) return fail(FDTDB_E_INVALID, "too many materials");
    return FDTDB_OK;
}

Material &new_material(fdtdb_grid_s *g, const fdtdb_box *box, int kind) {
    g->mats.emplace_back();
    Material &m = g->mats.back();
    m.kind = kind;
    m.mcells = 1;
    for (int a = 0; a < 3; a++) {
        m.lo[a] = box->lo[a];
        m.hi[a] = box->hi[a];
        m.mext[a] = (int)(box->hi[a] - box->lo[a]);
        m.mcells *= m.mext[a];
    }
    return m;
}

// CPML conductivity s(d) = s_max (d/L)^3, s_max = -4 ln(R0) / (2L); E nodes at integer
// positions, H nodes half a cell further along the axis.
double pml_sigma(const fdtdb_grid_s *g, int a, double pos) {
    if (g->bc[a] != FDTDB_BC_PML) return 0.0;
    const double L = (double)g->pml[a];
    const double smax = -4.0 * std::log(g->R0) / (2.0 * L);
    double d = 0.0;
    if (pos < L) d = L - pos;
    else if (pos > (double)(g->n[a] - 1) - L) d = pos - ((double)(g->n[a] - 1) - L);
    if (d <= 0.0) return 0.0;
    const double r = d / L;
    return smax * r * r * r;
}

// ---------------------------------------------------------------------------- region partition
// Split the grid into boxes of uniform update: cut at every material and CPML edge, then grow
// boxes greedily (z, then y, then x) over cuts of equal attributes.  E regions carry
// (material, CPML mask); H regions only the CPML mask (the H update is material-free).
//
// The absorbing layer of an axis starts where the grading is nonzero: E-type nodes at p < L and
// p > n-1-L, H-type nodes (half a cell further along) at p < L and p >= n-1-L.  In 3D with
// 4-aligned z layers the H regions are cut along z where the E regions are, and the region
// below the upper layer carries psi for its last 4-cell z group only (the node at n-1-L and
// three nodes where b = 1, c = 0 and psi stays exactly zero), in 4 slots per row: row splits
// then stay on 128-byte lines.  Otherwise, on the axis the vector kernels run along (z in 3D,
// y in 2D) the upper H cut is rounded down to a multiple of 32 cells for the same reason (a line
// shared by two regions is fetched and partially written by both); psi is again zero on the
// extra nodes.
bool z_tail_h(const fdtdb_grid_s *g) {
    return g->ndim == 3 && g->bc[2] == FDTDB_BC_PML && g->n[2] % 4 == 0 && g->pml[2] % 4 == 0 && !g->twin;
}

int upper_pml_cut(const fdtdb_grid_s *g, int a, bool h) {
    const int cut = (int)g->n[a] - g->pml[a];
    if (!h || (a == 2 && z_tail_h(g))) return cut;
    const bool vec_axis = (g->ndim == 3 && a == 2) || (g->ndim == 2 && a == 1);
    return std::max(g->pml[a], vec_axis ? (cut - 1) & ~31 : cut - 1);
}

// rows at each end of a Bloch axis that go into the wrap regions: one, or four along the axis the vector
// kernels run along (z in 3D, y in 2D) when its length is a multiple of 4, so that the regions between
// stay 4-aligned and take those kernels (only the end row reads the other part; the other three are
// updated as anywhere else)
int wrap_rows(const fdtdb_grid_s *g, int a) {
    const bool vec_axis = (g->ndim == 3 && a == 2) || (g->ndim == 2 && a == 1);
    return vec_axis && g->n[a] % 4 == 0 && g->n[a] >= 8 ? 4 : 1;
}

// a 2D Lorentz-Bath material on a Bloch pair that touches the wrap: its load-first kernel reads the other
// part in the wrap rows itself, so the whole material is one region that reads across the wrap rather than
// a region plus a one-row launch of the generic kernel (2048 x 1024 grid, N_b = 64: two 28 us launches a step)
bool bath_reads_wrap(const fdtdb_grid_s *g, const Material &m) {
    if (!g->twin || g->ndim != 2 || m.kind != K_BATH || m.ng <= 0 || m.ng > 16 || m.bext() || m.yfmt) return false;
    for (int a = 0; a < 2; a++)
        if (g->bph[a] != 0.0 && m.lo[a] == 0) return true;
    return false;
}

void partition(const fdtdb_grid_s *g, bool with_mats, std::vector<Region> &out) {
    const bool h = !with_mats;
    std::vector<int> br[3];
    int up[3] = {};
    for (int a = 0; a < 3; a++) {
        br[a].push_back(0);
        br[a].push_back(g->n[a]);
        if (g->bc[a] == FDTDB_BC_PML && a < g->ndim) {
            up[a] = upper_pml_cut(g, a, h);
            br[a].push_back(g->pml[a]);
            br[a].push_back(up[a]);
        }
        if (with_mats)
            for (auto &m : g->mats) {
                br[a].push_back((int)m.lo[a]);
                br[a].push_back((int)m.hi[a]);
            }
        if (g->twin && a < g->ndim && g->bph[a] != 0.0) br[a].push_back(h ? (int)g->n[a] - wrap_rows(g, a) : wrap_rows(g, a));
        std::sort(br[a].begin(), br[a].end());
        br[a].erase(std::unique(br[a].begin(), br[a].end()), br[a].end());
    }
    const int na = (int)br[0].size() - 1, nb = (int)br[1].size() - 1, nc = (int)br[2].size() - 1;
    // attribute of each atom: (mat, pml mask)
    std::vector<int> attr((size_t)na * nb * nc);
    std::map<std::pair<int, int>, int> ids;
    auto key = [&](int x, int y, int z) { return ((size_t)x * nb + y) * nc + z; };
    for (int x = 0; x < na; x++)
        for (int y = 0; y < nb; y++)
            for (int z = 0; z < nc; z++) {
                const int64_t lo[3] = {br[0][x], br[1][y], br[2][z]};
                const int64_t hi[3] = {br[0][x + 1], br[1][y + 1], br[2][z + 1]};
                int mat = -1;
                for (size_t mi = 0; with_mats && mi < g->mats.size(); mi++) {
                    const Material &m = g->mats[mi];
                    if (lo[0] >= m.lo[0] && lo[0] < m.hi[0] && lo[1] >= m.lo[1] && lo[1] < m.hi[1] && lo[2] >= m.lo[2] &&
                        lo[2] < m.hi[2])
                        mat = (int)mi;
                }
                int mask = 0;
                for (int a = 0; a < g->ndim; a++)
                    if (g->bc[a] == FDTDB_BC_PML && (lo[a] < g->pml[a] || lo[a] >= up[a])) mask |= 1 << a;
                for (int a = 0; g->twin && a < g->ndim; a++)     // bit 8: holds a row that reads across a Bloch axis
                    if (g->bph[a] != 0.0 && (h ? hi[a] == g->n[a] : lo[a] == 0)) mask |= 1 << 8;
                if (mat >= 0 && bath_reads_wrap(g, g->mats[mat])) mask |= 1 << 8;
                auto k = std::make_pair(mat, mask);
                if (!ids.count(k)) {
                    int id = (int)ids.size();
                    ids[k] = id;
                }
                attr[key(x, y, z)] = ids[k];
            }
    // greedy box growth: z first, then y, then x
    std::vector<char> used(attr.size(), 0);
    std::vector<std::pair<int, int>> rev(ids.size());
    for (auto &kv : ids) rev[kv.second] = kv.first;
    for (int x = 0; x < na; x++)
        for (int y = 0; y < nb; y++)
            for (int z = 0; z < nc; z++) {
                if (used[key(x, y, z)]) continue;
                const int id = attr[key(x, y, z)];
                int z1 = z + 1;
                while (z1 < nc && !used[key(x, y, z1)] && attr[key(x, y, z1)] == id) z1++;
                int y1 = y + 1;
                for (;; y1++) {
                    if (y1 >= nb) break;
                    bool ok = true;
                    for (int zz = z; zz < z1 && ok; zz++) ok = !used[key(x, y1, zz)] && attr[key(x, y1, zz)] == id;
                    if (!ok) break;
                }
                int x1 = x + 1;
                for (;; x1++) {
                    if (x1 >= na) break;
                    bool ok = true;
                    for (int yy = y; yy < y1 && ok; yy++)
                        for (int zz = z; zz < z1 && ok; zz++) ok = !used[key(x1, yy, zz)] && attr[key(x1, yy, zz)] == id;
                    if (!ok) break;
                }
                for (int xx = x; xx < x1; xx++)
                    for (int yy = y; yy < y1; yy++)
                        for (int zz = z; zz < z1; zz++) used[key(xx, yy, zz)] = 1;
                Region r;
                r.lo[0] = br[0][x]; r.hi[0] = br[0][x1];
                r.lo[1] = br[1][y]; r.hi[1] = br[1][y1];
                r.lo[2] = br[2][z]; r.hi[2] = br[2][z1];
                r.mat = rev[id].first;
                r.pml_mask = rev[id].second & 0xff;
                r.wrap = (rev[id].second >> 8) & 1;
                r.eps = r.mat >= 0 ? g->mats[r.mat].eps : 1.0;
                out.push_back(r);
            }
}

fdtdb_status build_regions(fdtdb_grid_s *g) {
    partition(g, true, g->regions);
    partition(g, false, g->hregions);
    if (z_tail_h(g) && g->pml[2] > 0)
        for (auto &r : g->hregions)
            if (r.hi[2] == (int)g->n[2] - g->pml[2] && !(r.pml_mask & (1 << 2))) {
                r.pml_mask |= 1 << 2;
                r.zlo = r.lo[2];
                r.zhi = std::max(r.lo[2], r.hi[2] - 4);
                r.zw = r.hi[2] - r.zhi;
            }
    // CPML psi storage per region, per component and curl term whose axis is absorbing
    for (int h = 0; h < 2; h++)
        for (auto &r : h ? g->hregions : g->regions) {
            if (!r.pml_mask) continue;
            for (int c = 0; c < 3; c++) {
                const int ax[2] = {curl_a1(c), curl_a2(c)};
                for (int t = 0; t < 2; t++) {
                    if (!(r.pml_mask & (1 << ax[t]))) continue;
                    const long long nc_ = r.psi_words(ax[t]);
                    if (!h && e_active(g->ndim, c)) TRY(g->alloc(&r.psiE[c][t], words(nc_, g->f64)));
                    if (h && h_active(g->ndim, c)) TRY(g->alloc(&r.psiH[c][t], words(nc_, g->f64)));
                }
            }
        }
    return FDTDB_OK;
}

bool region_hits_box(const Region &r, const int64_t *lo, const int64_t *hi) {
    for (int a = 0; a < 3; a++)
        if (r.hi[a] <= lo[a] || hi[a] <= r.lo[a]) return false;
    return true;
}

// algorithmic bytes per cell of a region's E and H launches: each state word read once and
// written once, neighbour values counted once
void region_bytes(const fdtdb_grid_s *g, const Region &r, double *be, double *bh) {
    const double w = g->f64 ? 8.0 : 4.0;
    int ne = 0, nh = 0;
    for (int c = 0; c < 3; c++) { ne += e_active(g->ndim, c); nh += h_active(g->ndim, c); }
    double e = (2.0 * ne + nh) * w, h = (ne + 2.0 * nh) * w;
    if (r.pml_mask) {
        int te = 0;
        double th = 0.0;
        for (int c = 0; c < 3; c++)
            for (int t = 0; t < 2; t++) {
                te += r.psiE[c][t] != nullptr;
                if (r.psiH[c][t]) th += (double)r.psi_words(t ? curl_a2(c) : curl_a1(c)) / (double)r.cells();
            }
        e += 2.0 * te * w;
        h += 2.0 * th * w;
    }
    if (r.mat >= 0) {
        const Material &m = g->mats[r.mat];
        if (m.kind == K_DRUDE) e += 2.0 * ne * w;
        else if (m.kind == K_BATH) e += 3.0 * ne * w + (m.sigma_per_cell ? w : 0.0) + 3.0 * ne * m.nb * (m.yfmt ? 2.0 : w);
        else if (m.kind == K_CLOSURE) e += 3.0 * ne * w + (m.sigma_per_cell ? w : 0.0) + 2.0 * ne * 16.0;
        else if (m.kind == K_MULTI)      // a Lorentz term reads two levels and writes one, a Drude term its increment
            for (int t = 0; t < m.nterm; t++) e += (m.coef[kCoefHead + kCoefMode * t + 5] != 0.0 ? 2.0 : 3.0) * ne * w;
    }
    *be = e;
    *bh = h;
}

fdtdb_status finalize(fdtdb_grid_s *g) {
    if (g->finalized) return FDTDB_OK;
    TRY(build_regions(g));
    // CPML coefficient tables: b = exp(-s dt), c = b - 1 at E-type and H-type positions
    for (int a = 0; a < 3; a++) {
        std::vector<double> b(g->n[a]), c(g->n[a]), bh(g->n[a]), ch(g->n[a]);
        for (int p = 0; p < g->n[a]; p++) {
            b[p] = std::exp(-pml_sigma(g, a, (double)p) * g->dt);
            c[p] = b[p] - 1.0;
            bh[p] = std::exp(-pml_sigma(g, a, (double)p + 0.5) * g->dt);
            ch[p] = bh[p] - 1.0;
        }
        TRY(g->alloc((void **)&g->pml_b[a], 8 * g->n[a]));
        TRY(g->alloc((void **)&g->pml_c[a], 8 * g->n[a]));
        TRY(g->alloc((void **)&g->pml_bh[a], 8 * g->n[a]));
        TRY(g->alloc((void **)&g->pml_ch[a], 8 * g->n[a]));
        HIP_TRY(hipMemcpy(g->pml_b[a], b.data(), 8 * g->n[a], hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g->pml_c[a], c.data(), 8 * g->n[a], hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g->pml_bh[a], bh.data(), 8 * g->n[a], hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g->pml_ch[a], ch.data(), 8 * g->n[a], hipMemcpyHostToDevice));
    }
    // sources
    std::vector<SourceDev> sd(g->srcs.size());
    for (size_t s = 0; s < g->srcs.size(); s++) {
        Source &S = g->srcs[s];
        SourceDev &d = sd[s];
        d.comp = S.comp;
        for (int a = 0; a < 3; a++) { d.lo[a] = (int)S.lo[a]; d.hi[a] = (int)S.hi[a]; }
        d.omega_c = S.omega_c;
        d.tau = 1.0 / S.width;
        d.t0 = 5.0 * d.tau;
        d.amplitude = S.amplitude;
        d.coef = g->dt / S.eps;
        d.profile = nullptr;
        if (!S.profile.empty()) {
            TRY(g->alloc((void **)&S.profile_dev, 8 * S.profile.size()));
            HIP_TRY(hipMemcpy(S.profile_dev, S.profile.data(), 8 * S.profile.size(), hipMemcpyHostToDevice));
            d.profile = S.profile_dev;
        }
    }
    TRY(g->alloc((void **)&g->src_dev, sizeof(SourceDev) * std::max<size_t>(1, sd.size())));
    if (!sd.empty()) HIP_TRY(hipMemcpy(g->src_dev, sd.data(), sizeof(SourceDev) * sd.size(), hipMemcpyHostToDevice));
    // launches: material regions alone; background E regions grouped; H regions grouped except
    // those the vectorized 3D kernel takes
    for (auto &r : g->regions)
        for (auto &e : g->ens)
            if (region_hits_box(r, e.lo, e.hi)) r.energy = true;
    for (auto &r : g->regions) {  // the sampling kernel reads the bath in the state type
        if (r.energy && r.mat >= 0 && g->mats[r.mat].yfmt)
            return fail(FDTDB_E_STATE, "an energy monitor covers a bath stored in 16 bits");
        if (r.energy && r.mat >= 0 && !g->mats[r.mat].lam.empty())
            return fail(FDTDB_E_STATE, "an energy monitor covers an anharmonic bath (its sum is the harmonic one)");
    }
    // threads of a region: one per cell, or (vector kernels) one per 4-cell group of the region's
    // fastest-axis range rounded out to whole groups
    auto blocks_of = [&](const Region &r, bool v4) {
        long long n = r.cells();
        if (v4) {
            const int a = g->ndim == 3 ? 2 : 1;
            n = n / (r.hi[a] - r.lo[a]) * (((r.hi[a] + 3) >> 2) - (r.lo[a] >> 2));
        }
        return (n + kBlock - 1) / kBlock;
    };
    auto make = [&](std::vector<Launch> &out, const std::vector<Region> &rs, const std::vector<int> &idx, bool group,
                    bool v4) {
        for (size_t s = 0; s < idx.size();) {
            Launch L;
            const size_t n = group ? std::min<size_t>(kMaxGroup, idx.size() - s) : 1;
            for (size_t q = 0; q < n; q++) {
                const Region &rg = rs[idx[s + q]];
                L.regs.push_back(idx[s + q]);
                L.pml |= rg.pml_mask != 0;
                L.energy |= rg.energy;
                L.blocks += blocks_of(rg, v4);
                L.cells += rg.cells();
            }
            L.grouped = n > 1;
            L.v4 = v4;
            out.push_back(L);
            s += n;
        }
    };
    // regions whose fastest-axis range (3D: z, 2D: y) is 4-aligned take the vectorized kernels
    auto z4 = [&](const Region &rg) {
        if (g->ndim == 2) return rg.lo[1] % 4 == 0 && (rg.hi[1] - rg.lo[1]) % 4 == 0 && g->n[1] % 4 == 0;
        return g->ndim == 3 && rg.lo[2] % 4 == 0 && (rg.hi[2] - rg.lo[2]) % 4 == 0 && g->n[2] % 4 == 0;
    };
    // 3D background regions without CPML terms may take the vector kernel unaligned: it computes
    // whole 4-cell groups and stores only the region's own cells at the edges
    auto bg_unaligned4 = [&](const Region &rg) {
        return g->ndim == 3 && g->n[2] % 4 == 0 && rg.mat < 0 && rg.pml_mask == 0;
    };
    {
        std::vector<int> bg4, bg, solo, drude4;
        for (int i = 0; i < (int)g->regions.size(); i++) {
            const Region &rg = g->regions[i];
            if (rg.mat >= 0) {
                const Material &mt = g->mats[rg.mat];
                const bool m4 = mt.mext[2] % 4 == 0 && (rg.lo[2] - (int)mt.lo[2]) % 4 == 0;
                (g->ndim == 3 && mt.kind == K_DRUDE && z4(rg) && m4 && !rg.energy && !rg.wrap ? drude4 : solo).push_back(i);
            } else if ((z4(rg) || bg_unaligned4(rg)) && !rg.energy && !rg.wrap) {   // wrap rows: generic kernels
                bg4.push_back(i);
            } else {
                bg.push_back(i);
            }
        }
        make(g->elaunch, g->regions, bg4, true, true);
        make(g->elaunch, g->regions, bg, bg.size() > 1, false);
        make(g->elaunch, g->regions, drude4, drude4.size() > 1, true);
        make(g->elaunch, g->regions, solo, false, false);
        std::vector<int> h4, hg;
        for (int i = 0; i < (int)g->hregions.size(); i++) {
            if (g->hregions[i].zw && !z4(g->hregions[i]))   // per-row psi slots: vector kernel only
                return fail(FDTDB_E_STATE, "H region with per-row psi slots but no 4-aligned z range");
            (z4(g->hregions[i]) && !g->hregions[i].wrap ? h4 : hg).push_back(i);
        }
        make(g->hlaunch, g->hregions, h4, true, true);
        make(g->hlaunch, g->hregions, hg, hg.size() > 1, false);
    }
    long long base = 0;
    for (auto &L : g->elaunch) {
        L.block_base = base;
        base += L.blocks;
    }
    g->total_blocks = base;
    for (int ph = 0; ph < 2; ph++)
        for (auto &L : ph ? g->hlaunch : g->elaunch) {
            if (!L.grouped && !L.v4) continue;
            const std::vector<Region> &rs = ph ? g->hregions : g->regions;
            RegionTable tab{};
            for (int s = 0; s < kMaxGroup; s++) tab.block0[s] = INT_MAX;
            int b0 = 0;
            for (size_t q = 0; q < L.regs.size(); q++) {
                const Region &rg = rs[L.regs[q]];
                RegionDesc &x = tab.d[q];
                for (int a = 0; a < 3; a++) { x.lo[a] = rg.lo[a]; x.ext[a] = rg.hi[a] - rg.lo[a]; }
                x.ext12 = x.ext[1] * x.ext[2];
                x.block0 = b0;
                tab.block0[q] = b0;
                b0 += (int)blocks_of(rg, L.v4);
                x.inv_eps = 1.0 / rg.eps;
                for (int c = 0; c < 3; c++)
                    for (int t = 0; t < 2; t++) x.psi[c][t] = ph ? rg.psiH[c][t] : rg.psiE[c][t];
                x.zlo = rg.zlo;
                x.zhi = rg.zhi;
                x.zw = rg.zw;
                if (ph == 0 && rg.mat >= 0 && g->mats[rg.mat].kind == K_DRUDE) {
                    const Material &mt = g->mats[rg.mat];
                    for (int c = 0; c < 3; c++) x.V[c] = mt.P[0][c];
                    for (int a = 0; a < 3; a++) { x.mlo[a] = (int)mt.lo[a]; x.mext[a] = mt.mext[a]; }
                    x.coef = mt.coef_dev;
                }
            }
            TRY(g->alloc((void **)&L.rd, sizeof(RegionTable)));
            HIP_TRY(hipMemcpy(L.rd, &tab, sizeof(RegionTable), hipMemcpyHostToDevice));
        }
    for (auto &e : g->ens) {
        e.nslots = base;
        TRY(g->alloc((void **)&e.partial, 24 * (size_t)base));
    }
    g->launches_per_step = 1 + (int)g->elaunch.size() + (int)g->hlaunch.size() + (int)g->ens.size() + (int)g->dfts.size();
    for (int ph = 0; ph < 2; ph++) {
        const std::vector<Launch> &ls = ph ? g->hlaunch : g->elaunch;
        const std::vector<Region> &rs = ph ? g->hregions : g->regions;
        for (size_t li = 0; li < ls.size(); li++) {
            const Launch &L = ls[li];
            const Region &r0 = rs[L.regs[0]];
            fdtdb_kernel_record k{};
            k.region = (int)li;
            k.phase = ph;
            k.kind = ph == 0 && r0.mat >= 0 ? g->mats[r0.mat].kind : K_BACKGROUND;
            k.n_bath = ph == 0 && r0.mat >= 0 ? g->mats[r0.mat].nb : 0;
            k.pml = L.pml;
            k.cells = L.cells;
            k.bytes = 0.0;
            for (int ri : L.regs) {
                double be, bh;
                region_bytes(g, rs[ri], &be, &bh);
                k.bytes += (ph == 0 ? be : bh) * (double)rs[ri].cells();
            }
            g->records.push_back(k);
        }
    }
    g->finalized = true;
    return FDTDB_OK;
}

void fill_fields(const fdtdb_grid_s *g, int *n, int *per) {
    for (int a = 0; a < 3; a++) {
        n[a] = g->n[a];
        per[a] = g->bc[a] == FDTDB_BC_PERIODIC ? 1 : 0;
    }
}

fdtdb_status ensure_energy_capacity(fdtdb_grid_s *g, long long last_step) {
    for (auto &e : g->ens) {
        const long long need = last_step / e.every + 1;
        if (need <= e.capacity) continue;
        long long cap = std::max<long long>(need, std::max<long long>(64, 2 * e.capacity));
        double *nw = nullptr;
        HIP_TRY(hipStreamSynchronize(g->stream));
        TRY(g->alloc((void **)&nw, 24 * (size_t)cap));
        if (e.out && e.capacity) HIP_TRY(hipMemcpy(nw, e.out, 24 * (size_t)e.capacity, hipMemcpyDeviceToDevice));
        e.out = nw;   // the old buffer stays in the grid's allocation list until destroy
        e.capacity = cap;
        if (g->graph) {   // captured launches hold the old buffer
            (void)hipGraphExecDestroy(g->graph);
            g->graph = nullptr;
        }
    }
    return FDTDB_OK;
}

fdtdb_status flush_dft(fdtdb_grid_s *g, Dft &d) {
    if (d.nstaged == 0) return FDTDB_OK;
    HIP_TRY(launch_dft_flush(g->clock, d.omega_dev, d.nf, d.nstaged, g->dt, d.tw, d.stage, d.npts, d.acc, g->stream));
    d.nstaged = 0;
    return FDTDB_OK;
}

hipEvent_t take_event(fdtdb_grid_s *g) {
    if (!g->pool.empty()) {
        hipEvent_t e = g->pool.back();
        g->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

fdtdb_status collect_events(fdtdb_grid_s *g) {
    if (g->pending.empty()) return FDTDB_OK;
    HIP_TRY(hipStreamSynchronize(g->stream));
    for (auto &p : g->pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        g->records[p.rec].ms_total += ms;
        g->records[p.rec].launches += 1;
        g->pool.push_back(p.a);
        g->pool.push_back(p.b);
    }
    g->pending.clear();
    return FDTDB_OK;
}

// enqueue one full step (no host synchronization)
// cos phi_a and (part 0: -sin phi_a, part 1: +sin phi_a) of every axis of a Bloch pair
void bloch_coefs(const fdtdb_grid_s *g, double *bc, double *bs) {
    for (int ax = 0; ax < 3; ax++) {
        bc[ax] = std::cos(g->bph[ax]);
        bs[ax] = (g->part == 0 ? -1.0 : 1.0) * std::sin(g->bph[ax]);
    }
}

// the E half of a step: clock, E and material launches, energy sums, probes
fdtdb_status enqueue_e(fdtdb_grid_s *g) {
    const long long n = g->steps;
    const int cur = (int)(n & 1), nxt = cur ^ 1;
    HIP_TRY(launch_tick(g->clock, g->src_dev, (int)g->srcs.size(), g->dt, g->stream));
    for (auto &L : g->elaunch) {
        const Region &r = g->regions[L.regs[0]];
        EArgs a{};
        for (int c = 0; c < 3; c++) { a.E[c] = g->E[c]; a.H[c] = g->H[c]; }
        bool wrap = false;
        for (int ri : L.regs) wrap |= g->regions[ri].wrap;
        if (g->twin && wrap) {              // only launches over wrap rows read the other part
            a.bloch = 1;
            for (int c = 0; c < 3; c++) a.Htw[c] = g->twin->H[c];
            bloch_coefs(g, a.bcos, a.bsin);
        }
        fill_fields(g, a.n, a.per);
        for (int ax = 0; ax < 3; ax++) { a.lo[ax] = r.lo[ax]; a.ext[ax] = r.hi[ax] - r.lo[ax]; }
        a.ext12 = a.ext[1] * a.ext[2];
        a.dt = g->dt;
        a.inv_eps = 1.0 / r.eps;
        if (L.grouped || L.v4) {
            for (int ax = 0; ax < 3; ax++) { a.lo[ax] = 0; a.ext[ax] = 1; }
            a.ext[0] = (int)(L.blocks * kBlock);
            a.ext12 = 1;
            a.rd = L.rd;
            a.nrd = L.v4 ? -(int)L.regs.size() : (int)L.regs.size();
        }
        int kind = K_BACKGROUND, ng = 0;
        for (int c = 0; c < 3; c++)
            for (int t = 0; t < 2; t++) a.psi[c][t] = r.psiE[c][t];
        for (int ax = 0; ax < 3; ax++) { a.pml_b[ax] = g->pml_b[ax]; a.pml_c[ax] = g->pml_c[ax]; }
        if (r.mat >= 0) {
            Material &m = g->mats[r.mat];
            kind = m.kind;
            ng = m.ng;
            for (int ax = 0; ax < 3; ax++) { a.mlo[ax] = (int)m.lo[ax]; a.mext[ax] = m.mext[ax]; }
            a.mcells = m.mcells;
            if (kind == K_DRUDE) {
                for (int c = 0; c < 3; c++) a.Pcur[c] = m.P[0][c];
            } else if (kind == K_MULTI) {
                for (int c = 0; c < 3; c++) {
                    a.Pcur[c] = m.P[cur][c];
                    a.Pnew[c] = m.P[nxt][c];
                }
                a.nterm = m.nterm;
                a.drude_mask = 0;
                for (int t = 0; t < m.nterm; t++)
                    if (m.coef[kCoefHead + kCoefMode * t + 5] != 0.0) a.drude_mask |= 1 << t;
            } else if (kind == K_BATH || kind == K_CLOSURE) {
                for (int c = 0; c < 3; c++) {
                    a.Pcur[c] = m.P[cur][c];
                    a.Pnew[c] = m.P[nxt][c];
                    a.Ycur[c] = m.Y[cur][c];
                    a.Ynew[c] = m.Y[nxt][c];
                    a.hid[c] = m.hid[c];
                }
                a.cw = m.cw_dev;
                for (int q = 0; q < 4; q++) a.cscale[q] = m.cscale[q];
                a.yfmt = m.yfmt;
                a.yscale = m.yscale;
                a.yinv = 1.0 / m.yscale;
                a.nb = m.nb;
                a.bext = kind == K_BATH ? m.bext() : 0;
                a.key0 = (unsigned)m.seed;
                a.key1 = (unsigned)(m.seed >> 32);
            }
            a.sigma = m.sigma_per_cell ? m.sigma_dev : nullptr;
            a.sigma0 = m.sigma0;
            a.coef = m.coef_dev;
        }
        a.clock = g->clock;
        a.nsrc = (int)g->srcs.size();
        for (int s = 0; s < a.nsrc; s++) {
            const Source &S = g->srcs[s];
            SourceArg &d = a.src[s];
            d.comp = S.comp;
            for (int ax = 0; ax < 3; ax++) { d.lo[ax] = (int)S.lo[ax]; d.hi[ax] = (int)S.hi[ax]; }
            d.coef = g->dt / S.eps;
            d.profile = S.profile_dev;
        }
        a.nen = 0;
        if (L.energy) {
            for (auto &e : g->ens) {
                EnergyDev &d = a.en[a.nen++];
                for (int ax = 0; ax < 3; ax++) { d.lo[ax] = (int)e.lo[ax]; d.hi[ax] = (int)e.hi[ax]; }
                d.every = e.every;
                d.partial = e.partial;
            }
        }
        a.block_base = L.block_base;
        const int rec = (int)(&L - &g->elaunch[0]);
        Pending pe{rec, nullptr, nullptr};
        const bool ev = g->profiling == 1 || (g->profiling == 2 && (kind == K_BATH || kind == K_CLOSURE));
        if (ev) {
            pe.a = take_event(g);
            pe.b = take_event(g);
            if (!pe.a || !pe.b) return fail(FDTDB_E_DEVICE, "event creation failed");
            HIP_TRY(hipEventRecord(pe.a, g->stream));
        }
        const double *ch = r.mat >= 0 && !g->mats[r.mat].coef.empty() ? g->mats[r.mat].coef.data() : nullptr;
        HIP_TRY(launch_update_e(g->ndim, g->f64, a, ch, kind, ng, L.pml, L.energy, g->stream));
        if (ev) {
            HIP_TRY(hipEventRecord(pe.b, g->stream));
            g->pending.push_back(pe);
        }
    }
    for (auto &e : g->ens)
        HIP_TRY(launch_energy_reduce(g->clock, e.partial, e.nslots, e.every, e.out, e.capacity, g->stream));
    for (auto &pr : g->probes)
        HIP_TRY(launch_probe(g->f64, g->E[pr.comp], g->mats[pr.mat].P[nxt][pr.comp], pr.q, pr.m, pr.n, g->clock,
                             pr.capacity, pr.E, pr.P, g->stream));
    return FDTDB_OK;
}

// the H half of a step
fdtdb_status enqueue_h(fdtdb_grid_s *g) {
    for (auto &L : g->hlaunch) {
        const Region &r = g->hregions[L.regs[0]];
        HArgs a{};
        for (int c = 0; c < 3; c++) { a.E[c] = g->E[c]; a.H[c] = g->H[c]; }
        bool wrap = false;
        for (int ri : L.regs) wrap |= g->hregions[ri].wrap;
        if (g->twin && wrap) {
            for (int c = 0; c < 3; c++) a.Etw[c] = g->twin->E[c];
            bloch_coefs(g, a.bcos, a.bsin);
        }
        fill_fields(g, a.n, a.per);
        for (int ax = 0; ax < 3; ax++) { a.lo[ax] = r.lo[ax]; a.ext[ax] = r.hi[ax] - r.lo[ax]; }
        a.ext12 = a.ext[1] * a.ext[2];
        a.dt = g->dt;
        for (int c = 0; c < 3; c++)
            for (int t = 0; t < 2; t++) a.psi[c][t] = r.psiH[c][t];
        for (int ax = 0; ax < 3; ax++) { a.pml_b[ax] = g->pml_bh[ax]; a.pml_c[ax] = g->pml_ch[ax]; }
        if (L.grouped || L.v4) {
            for (int ax = 0; ax < 3; ax++) { a.lo[ax] = 0; a.ext[ax] = 1; }
            a.ext[0] = (int)(L.blocks * kBlock);
            a.ext12 = 1;
            a.rd = L.rd;
            a.nrd = L.v4 ? -(int)L.regs.size() : (int)L.regs.size();
        }
        const int rec = (int)g->elaunch.size() + (int)(&L - &g->hlaunch[0]);
        Pending pe{rec, nullptr, nullptr};
        if (g->profiling == 1) {
            pe.a = take_event(g);
            pe.b = take_event(g);
            if (!pe.a || !pe.b) return fail(FDTDB_E_DEVICE, "event creation failed");
            HIP_TRY(hipEventRecord(pe.a, g->stream));
        }
        HIP_TRY(launch_update_h(g->ndim, g->f64, a, L.pml, g->stream));
        if (g->profiling == 1) {
            HIP_TRY(hipEventRecord(pe.b, g->stream));
            g->pending.push_back(pe);
        }
    }
    return FDTDB_OK;
}

// the monitors' DFT staging of a step, and the step count
fdtdb_status enqueue_dft(fdtdb_grid_s *g) {
    for (auto &d : g->dfts) {
        DftArgs a{};
        a.axis = d.axis;
        a.npts = d.npts;
        for (int ax = 0; ax < 3; ax++) { a.lo[ax] = (int)d.lo[ax]; a.ext[ax] = (int)(d.hi[ax] - d.lo[ax]); }
        a.ext12 = a.ext[1] * a.ext[2];
        fill_fields(g, a.n, a.per);
        a.E[0] = g->E[d.t1]; a.E[1] = g->E[d.t2];
        a.H[0] = g->H[d.t1]; a.H[1] = g->H[d.t2];
        a.stage = d.stage;
        a.slot = d.nstaged;
        HIP_TRY(launch_dft_stage(g->f64, a, g->stream));
        d.nstaged++;
        if (d.nstaged == kDftSlots) TRY(flush_dft(g, d));
    }
    g->steps++;
    return FDTDB_OK;
}

fdtdb_status enqueue_step(fdtdb_grid_s *g) {
    TRY(enqueue_e(g));
    TRY(enqueue_h(g));
    return enqueue_dft(g);
}

// one step of a Bloch pair (both parts on one stream): each half step runs on both parts before the next
// half step, so that the reads across a Bloch axis see the other part at the same time level
fdtdb_status enqueue_pair_step(fdtdb_grid_s *re) {
    fdtdb_grid_s *im = re->twin;
    TRY(enqueue_e(re));
    TRY(enqueue_e(im));
    TRY(enqueue_h(re));
    TRY(enqueue_h(im));
    TRY(enqueue_dft(re));
    return enqueue_dft(im);
}

fdtdb_status sync(fdtdb_grid_s *g) {
    HIP_TRY(hipStreamSynchronize(g->stream));
    return FDTDB_OK;
}

fdtdb_status flush_all(fdtdb_grid_s *g) {
    for (auto &d : g->dfts) TRY(flush_dft(g, d));
    return FDTDB_OK;
}

// copy a device array of the storage type to host doubles
fdtdb_status read_state(fdtdb_grid_s *g, const void *src, long long n, double *out) {
    if (!src) {
        std::fill(out, out + n, 0.0);
        return FDTDB_OK;
    }
    if (g->f64) {
        HIP_TRY(hipMemcpy(out, src, 8 * (size_t)n, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp((size_t)n);
        HIP_TRY(hipMemcpy(tmp.data(), src, 4 * (size_t)n, hipMemcpyDeviceToHost));
        for (long long i = 0; i < n; i++) out[i] = tmp[i];
    }
    return FDTDB_OK;
}

fdtdb_status write_state(fdtdb_grid_s *g, void *dst, long long n, const double *in) {
    if (g->f64) {
        HIP_TRY(hipMemcpy(dst, in, 8 * (size_t)n, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp((size_t)n);
        for (long long i = 0; i < n; i++) tmp[i] = (float)in[i];
        HIP_TRY(hipMemcpy(dst, tmp.data(), 4 * (size_t)n, hipMemcpyHostToDevice));
    }
    return FDTDB_OK;
}

}  // namespace

// ============================================================================ C ABI
// ---------------------------------------------------------------------------- device memory
namespace {
std::mutex g_mem_mu;
DevAllocator g_mem{nullptr, nullptr, nullptr};
}  // namespace

DevAllocator fdtdb::current_allocator() {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    return g_mem;
}

hipError_t fdtdb::dev_alloc(const DevAllocator &a, void **p, size_t bytes) {
    if (!a.alloc) return hipMalloc(p, bytes);
    *p = a.alloc(bytes, a.ctx);
    if (!*p) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(*p) % 256 != 0) {   // the kernels' vector accesses assume it
        a.free(*p, a.ctx);
        *p = nullptr;
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}

void fdtdb::dev_free(const DevAllocator &a, void *p) {
    if (!p) return;
    if (a.free) a.free(p, a.ctx);
    else (void)hipFree(p);
}

// ---------------------------------------------------------------------------- checkpoint
namespace {

constexpr char kStateMagic[8] = {'F', 'D', 'T', 'D', 'B', 'S', 'T', '1'};

// FNV-1a over the set-up of the grid: two grids with the same fingerprint have the same state
// buffers with the same meaning
struct Fnv {
    uint64_t h = 1469598103934665603ULL;
    void bytes(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; i++) { h ^= c[i]; h *= 1099511628211ULL; }
    }
    template <class T> void v(const T &x) { bytes(&x, sizeof x); }
    void vec(const std::vector<double> &x) { v(x.size()); if (!x.empty()) bytes(x.data(), 8 * x.size()); }
};

uint64_t fingerprint(const fdtdb_grid_s *g) {
    Fnv f;
    f.v(g->ndim); f.bytes(g->n, sizeof g->n); f.v(g->dt); f.v(g->R0); f.v(g->f64);
    f.bytes(g->bc, sizeof g->bc); f.bytes(g->pml, sizeof g->pml);
    f.v(g->twin != nullptr); f.v(g->part); f.bytes(g->bph, sizeof g->bph);
    f.v(g->mats.size());
    for (auto &m : g->mats) {
        f.v(m.kind); f.bytes(m.lo, sizeof m.lo); f.bytes(m.hi, sizeof m.hi); f.v(m.eps); f.v(m.omega0);
        f.v(m.gamma0); f.v(m.sigma0); f.v(m.sigma_per_cell); f.v(m.nb); f.vec(m.wj); f.vec(m.gj); f.vec(m.kj);
        f.vec(m.coef); f.v(m.cw_dev != nullptr); f.bytes(m.cscale, sizeof m.cscale);
        f.v(m.sigma_hash); f.v(m.weight_hash); f.v(m.nterm); f.v(m.yfmt); f.v(m.yscale);
        f.v(m.kT); f.v(m.seed); f.vec(m.lam);
    }
    f.v(g->srcs.size());
    for (auto &x : g->srcs) {
        f.v(x.comp); f.bytes(x.lo, sizeof x.lo); f.bytes(x.hi, sizeof x.hi); f.v(x.omega_c); f.v(x.width);
        f.v(x.amplitude); f.vec(x.profile);
    }
    f.v(g->dfts.size());
    for (auto &d : g->dfts) { f.v(d.axis); f.bytes(d.lo, sizeof d.lo); f.bytes(d.hi, sizeof d.hi); f.vec(d.omega); }
    f.v(g->ens.size());
    for (auto &e : g->ens) { f.bytes(e.lo, sizeof e.lo); f.bytes(e.hi, sizeof e.hi); f.v(e.every); }
    f.v(g->probes.size());
    for (auto &p : g->probes) { f.v(p.mat); f.v(p.comp); f.v(p.n); f.v(p.capacity); }
    return f.h;
}

// every device buffer whose contents evolve with the steps, in a fixed order; energy sample
// buffers only up to the samples taken in the first `steps` steps
fdtdb_status state_buffers(const fdtdb_grid_s *g, long long steps, std::vector<std::pair<void *, size_t>> &out) {
    auto add = [&](void *p) -> fdtdb_status {
        if (!p) return FDTDB_OK;
        auto it = g->sizes.find(p);
        if (it == g->sizes.end()) return fail(FDTDB_E_STATE, "state buffer without a recorded size");
        out.emplace_back(p, it->second);
        return FDTDB_OK;
    };
    out.emplace_back(g->clock, sizeof(Clock));
    for (int c = 0; c < 3; c++) { TRY(add(g->E[c])); TRY(add(g->H[c])); }
    for (auto &m : g->mats) {
        for (int l = 0; l < 2; l++)
            for (int c = 0; c < 3; c++) { TRY(add(m.P[l][c])); TRY(add(m.Y[l][c])); }
        for (int c = 0; c < 3; c++) TRY(add(m.hid[c]));
    }
    for (int h = 0; h < 2; h++)
        for (auto &r : h ? g->hregions : g->regions)
            for (int c = 0; c < 3; c++)
                for (int t = 0; t < 2; t++) TRY(add(h ? r.psiH[c][t] : r.psiE[c][t]));
    for (auto &d : g->dfts) { TRY(add(d.stage)); TRY(add(d.acc)); }
    for (auto &e : g->ens) {
        const long long n = steps == 0 ? 0 : (steps - 1) / e.every + 1;
        if (n > e.capacity) return fail(FDTDB_E_STATE, "energy buffer smaller than its samples");
        if (n > 0) out.emplace_back(e.out, 24 * (size_t)n);
    }
    for (auto &p : g->probes) { TRY(add(p.E)); TRY(add(p.P)); }
    return FDTDB_OK;
}

struct File {
    FILE *f = nullptr;
    ~File() { if (f) fclose(f); }
};

}  // namespace

extern "C" {

const char *fdtdb_last_error(void) { return g_err.c_str(); }
const char *fdtdb_version(void) { return "fdtdb 0.1 (gfx950)"; }

fdtdb_status fdtdb_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(FDTDB_E_INVALID, "allocator needs both alloc and free");
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem = DevAllocator{alloc, free_fn, alloc ? ctx : nullptr};
    return FDTDB_OK;
}

fdtdb_status fdtdb_create_grid(const fdtdb_grid_desc *d, fdtdb_grid *out) {
    if (!d || !out) return fail(FDTDB_E_INVALID, "null argument");
    *out = nullptr;
    if (d->ndim < 1 || d->ndim > 3) return fail(FDTDB_E_INVALID, "ndim must be 1, 2 or 3");
    if (!(d->courant > 0.0)) return fail(FDTDB_E_INVALID, "courant must be > 0");
    if (d->courant > 1.0 / std::sqrt((double)d->ndim) + 1e-15)
        return fail(FDTDB_E_UNSTABLE, "courant %.6g exceeds the vacuum limit 1/sqrt(%d)", d->courant, d->ndim);
    if (d->dtype != FDTDB_F32 && d->dtype != FDTDB_F64) return fail(FDTDB_E_INVALID, "bad dtype");
    long long total = 1;
    for (int a = 0; a < 3; a++) {
        long long na = a < d->ndim ? d->n[a] : 1;
        if (na < 1 || na > (1 << 30)) return fail(FDTDB_E_INVALID, "bad extent on axis %d", a);
        total *= na;
    }
    if (total >= (1LL << 31)) return fail(FDTDB_E_INVALID, "grid too large (%lld cells)", total);
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(FDTDB_E_DEVICE, "no HIP device: %s", hipGetErrorString(he));
    auto *g = new fdtdb_grid_s();
    g->ndim = d->ndim;
    for (int a = 0; a < 3; a++) {
        g->n[a] = a < d->ndim ? (int)d->n[a] : 1;
        g->bc[a] = a < d->ndim ? (int)d->bc[a] : FDTDB_BC_PERIODIC;
        if (g->bc[a] < 0 || g->bc[a] > 2) { delete g; return fail(FDTDB_E_INVALID, "bad boundary on axis %d", a); }
        g->pml[a] = g->bc[a] == FDTDB_BC_PML ? d->pml_cells[a] : 0;
        if (g->bc[a] == FDTDB_BC_PML && (g->pml[a] < 1 || 2 * g->pml[a] >= g->n[a])) {
            delete g;
            return fail(FDTDB_E_INVALID, "bad CPML thickness on axis %d", a);
        }
    }
    g->ncell = total;
    g->dt = d->courant;
    g->R0 = d->pml_R0 > 0 ? d->pml_R0 : 1e-8;
    g->f64 = d->dtype == FDTDB_F64;
    if (d->hip_stream) {
        g->stream = (hipStream_t)d->hip_stream;
    } else {
        he = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (he != hipSuccess) { delete g; return fail(FDTDB_E_DEVICE, "stream: %s", hipGetErrorString(he)); }
        g->own_stream = true;
    }
    fdtdb_status st = FDTDB_OK;
    for (int c = 0; c < 3 && st == FDTDB_OK; c++) {
        // the six field arrays are handed out 0, 1, ..., 5 KiB into their allocations: on the 512^3
        // grid the H pass took 1.006 ms against 1.018 ms, the background E pass 0.806 against 0.816 ms
        if (e_active(g->ndim, c)) st = g->alloc(&g->E[c], words(total, g->f64), 1024 * (size_t)c);
        if (st == FDTDB_OK && h_active(g->ndim, c)) st = g->alloc(&g->H[c], words(total, g->f64), 1024 * (size_t)(3 + c));
    }
    if (st == FDTDB_OK) st = g->alloc((void **)&g->clock, sizeof(Clock));
    if (st == FDTDB_OK) st = g->alloc((void **)&g->flag_dev, sizeof(int));
    if (st != FDTDB_OK) {
        std::string msg = g_err;
        fdtdb_destroy_grid(g);
        g_err = msg;
        return st;
    }
    *out = g;
    return FDTDB_OK;
}

fdtdb_status fdtdb_destroy_grid(fdtdb_grid g) {
    if (!g) return FDTDB_OK;
    if (g->twin) {
        if (g->own_stream && g->twin->stream == g->stream) {   // the other part keeps the shared stream
            g->twin->own_stream = true;
            g->own_stream = false;
        }
        g->twin->twin = nullptr;
        g->twin->orphan = true;
    }
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->graph) (void)hipGraphExecDestroy(g->graph);
    for (auto &p : g->pending) { g->pool.push_back(p.a); g->pool.push_back(p.b); }
    for (hipEvent_t e : g->pool) (void)hipEventDestroy(e);
    for (void *p : g->allocs) dev_free(g->mem, p);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_eps_inf(fdtdb_grid g, const fdtdb_box *box, double eps_inf, int *material_id) {
    TRY(check_new_material(g, box, false));
    if (!(eps_inf > 0.0) || !std::isfinite(eps_inf)) return fail(FDTDB_E_INVALID, "eps_inf must be > 0");
    Material &m = new_material(g, box, K_BACKGROUND);
    m.eps = eps_inf;
    if (material_id) *material_id = (int)g->mats.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_drude(fdtdb_grid g, const fdtdb_box *box, double omega_p, double gamma, double eps_inf,
                             int *material_id) {
    TRY(check_new_material(g, box, true));
    if (!(eps_inf > 0.0) || !(omega_p >= 0.0) || !(gamma >= 0.0))
        return fail(FDTDB_E_INVALID, "Drude needs eps_inf > 0, omega_p >= 0, gamma >= 0");
    const double dt = g->dt;
    // lossless lattice bound: eps 4/dt^2 - wp^2 - 4 ndim >= 0
    const double margin = eps_inf * 4.0 / (dt * dt) - omega_p * omega_p - 4.0 * g->ndim;
    if (margin < 0.0)
        return fail(FDTDB_E_UNSTABLE, "Drude medium unstable: need eps_inf >= %.6g", dt * dt * (omega_p * omega_p + 4.0 * g->ndim) / 4.0);
    Material &m = new_material(g, box, K_DRUDE);
    m.eps = eps_inf;
    m.omega0 = omega_p;
    m.gamma0 = gamma;
    const double gg = 0.5 * gamma * dt;
    m.coef.assign(kCoefHead, 0.0);
    m.coef[0] = omega_p * omega_p * dt * dt / (1.0 + gg);
    m.coef[1] = (1.0 - gg) / (1.0 + gg);
    m.coef[2] = omega_p > 0 ? 1.0 / (omega_p * omega_p) : 0.0;
    TRY(g->alloc((void **)&m.coef_dev, 8 * m.coef.size()));
    HIP_TRY(hipMemcpy(m.coef_dev, m.coef.data(), 8 * m.coef.size(), hipMemcpyHostToDevice));
    for (int c = 0; c < 3; c++)
        if (e_active(g->ndim, c)) TRY(g->alloc(&m.P[0][c], words(m.mcells, g->f64)));
    if (material_id) *material_id = (int)g->mats.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_multi_term(fdtdb_grid g, const fdtdb_box *box, double eps_inf, int n_terms, const int *kinds,
                                  const double *omega, const double *gamma, const double *sigma, int *material_id) {
    TRY(check_new_material(g, box, true));
    if (!(eps_inf > 0.0) || n_terms < 1 || n_terms > kMaxTerms || !kinds || !omega || !gamma || !sigma)
        return fail(FDTDB_E_INVALID, "multi-term material needs eps_inf > 0 and 1..%d terms", kMaxTerms);
    const double dt = g->dt, X = 4.0 / (dt * dt);
    double e = eps_inf;
    for (int p = 0; p < n_terms; p++) {
        if ((kinds[p] != 0 && kinds[p] != 1) || !(omega[p] > 0.0) || !(gamma[p] >= 0.0) ||
            (kinds[p] == 0 && !(sigma[p] > 0.0)))
            return fail(FDTDB_E_INVALID, "term %d: kind 0 (Lorentz: omega0, gamma, sigma > 0) or 1 (Drude: omega_p, gamma)", p);
        if (omega[p] * dt >= 2.0) return fail(FDTDB_E_UNSTABLE, "term %d: omega dt >= 2", p);
        const double w2 = omega[p] * omega[p];
        e += kinds[p] == 1 ? -w2 / X : w2 * sigma[p] / (w2 - X);
    }
    // lossless lattice bound: the largest mode frequency X = s^2 of X (eps_inf + sum_p chi_p(X)) = 4 ndim stays
    // below 4/dt^2 (the branch above every resonance increases, so its value at X = 4/dt^2 decides)
    if (X * e - 4.0 * g->ndim < 0.0)
        return fail(FDTDB_E_UNSTABLE, "multi-term medium violates the lattice stability bound (margin %.6g)",
                    X * e - 4.0 * g->ndim);
    Material &m = new_material(g, box, K_MULTI);
    m.eps = eps_inf;
    m.nterm = n_terms;
    m.coef.assign(kCoefHead + kCoefMode * n_terms, 0.0);
    for (int p = 0; p < n_terms; p++) {
        const double w2 = omega[p] * omega[p], A = 1.0 + 0.5 * gamma[p] * dt;
        double *t = &m.coef[kCoefHead + kCoefMode * p];
        const bool drude = kinds[p] == 1;
        // Lorentz: eq:Pz_1D_Lorentz; Drude: the same with omega0^2 dropped, written for the increment
        // V = P^{n+1/2} - P^{n-1/2}: V' = (w_p^2 dt^2 E + (1 - g dt/2) V) / (1 + g dt/2)
        t[0] = w2 * dt * dt / A;                                   // times sigma (t[6]) for a Lorentz term
        t[1] = drude ? (1.0 - 0.5 * gamma[p] * dt) / A : (w2 * dt * dt - 2.0) / A;
        t[2] = drude ? 0.0 : (1.0 - 0.5 * gamma[p] * dt) / A;
        t[3] = drude ? 1.0 / w2 : 1.0 / (sigma[p] * w2);           // rho of the term's energy
        t[4] = drude ? 0.0 : w2;
        t[5] = kinds[p];
        t[6] = drude ? 1.0 : sigma[p];
    }
    TRY(g->alloc((void **)&m.coef_dev, 8 * m.coef.size()));
    HIP_TRY(hipMemcpy(m.coef_dev, m.coef.data(), 8 * m.coef.size(), hipMemcpyHostToDevice));
    for (int lvl = 0; lvl < 2; lvl++)
        for (int c = 0; c < 3; c++)
            if (e_active(g->ndim, c)) TRY(g->alloc(&m.P[lvl][c], words(m.mcells * n_terms, g->f64)));
    if (material_id) *material_id = (int)g->mats.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_lorentz_bath(fdtdb_grid g, const fdtdb_box *box, double omega0, double gamma0,
                                    double eps_inf, const double *sigma_cells, double sigma_uniform, int n_bath,
                                    const double *omega_j, const double *gamma_j, const double *k_j,
                                    int *material_id) {
    TRY(check_new_material(g, box, true));
    if (!(eps_inf > 0.0) || !(omega0 > 0.0) || !(gamma0 >= 0.0) || n_bath < 0 || n_bath > 64)
        return fail(FDTDB_E_INVALID, "Lorentz-Bath needs eps_inf > 0, omega0 > 0, gamma0 >= 0, 0 <= n_bath <= 64");
    if (n_bath > 0 && (!omega_j || !gamma_j || !k_j)) return fail(FDTDB_E_INVALID, "bath arrays missing");
    const double dt = g->dt;
    long long mc = 1;
    for (int a = 0; a < 3; a++) mc *= box->hi[a] - box->lo[a];
    double smax = sigma_uniform;
    if (sigma_cells) {
        smax = 0.0;
        for (long long q = 0; q < mc; q++) {
            if (!(sigma_cells[q] > 0.0) || !std::isfinite(sigma_cells[q]))
                return fail(FDTDB_E_INVALID, "sigma must be > 0 in every cell");
            smax = std::max(smax, sigma_cells[q]);
        }
    } else if (!(sigma_uniform > 0.0)) {
        return fail(FDTDB_E_INVALID, "sigma must be > 0");
    }
    if (omega0 * dt >= 2.0) return fail(FDTDB_E_UNSTABLE, "omega0 dt >= 2");
    const double w02 = omega0 * omega0;
    const double margin = eps_inf * (4.0 / (dt * dt) - w02) - w02 * smax - 4.0 * g->ndim * (1.0 - w02 * dt * dt / 4.0);
    if (margin < 0.0) return fail(FDTDB_E_UNSTABLE, "Lorentz medium violates the lattice stability bound (margin %.6g)", margin);
    for (int jb = 0; jb < n_bath; jb++) {
        if (!(omega_j[jb] > 0.0) || omega_j[jb] * dt >= 2.0 || !(gamma_j[jb] >= 0.0) || !std::isfinite(k_j[jb]))
            return fail(FDTDB_E_UNSTABLE, "bath mode %d: need 0 < omega_j dt < 2, gamma_j >= 0", jb);
    }
    Material &m = new_material(g, box, K_BATH);
    m.eps = eps_inf;
    m.omega0 = omega0;
    m.gamma0 = gamma0;
    m.sigma0 = sigma_uniform;
    m.sigma_max = smax;
    m.nb = n_bath;
    // groups of four modes; pad to a supported count with uncoupled modes (k = 0 keeps them at zero)
    int ng = (n_bath + 3) / 4;
    static const int supported[] = {0, 1, 2, 3, 4, 6, 8, 12, 16};
    for (int s : supported)
        if (s >= ng) { ng = s; break; }
    m.ng = ng;
    m.wj.assign(omega_j, omega_j + n_bath);
    m.gj.assign(gamma_j, gamma_j + n_bath);
    m.kj.assign(k_j, k_j + n_bath);
    // coefficient table (FP64): eq:Pz_update-LB and eq:Yzj_finite_difference
    double skc = 0.0;
    std::vector<double> aj(4 * ng, 0.0), bj(4 * ng, 0.0), cj(4 * ng, 0.0), kk(4 * ng, 0.0), w2(4 * ng, 0.0);
    for (int jb = 0; jb < n_bath; jb++) {
        const double den = 1.0 + 0.5 * gamma_j[jb] * dt;
        aj[jb] = (2.0 - omega_j[jb] * omega_j[jb] * dt * dt) / den;
        bj[jb] = -2.0 / den;
        cj[jb] = k_j[jb] * dt / (2.0 * den);
        kk[jb] = k_j[jb];
        w2[jb] = omega_j[jb] * omega_j[jb];
        skc += k_j[jb] * cj[jb];
    }
    const double A = 1.0 + 0.5 * gamma0 * dt + 0.5 * dt * skc;
    m.coef.assign(kCoefHead + kCoefMode * 4 * ng, 0.0);
    m.coef[0] = w02 * dt * dt / A;
    m.coef[1] = (w02 * dt * dt - 2.0) / A;
    m.coef[2] = (1.0 - 0.5 * gamma0 * dt - 0.5 * dt * skc) / A;
    m.coef[3] = 1.0 / w02;
    m.coef[4] = w02;
    m.coef[5] = 1.0 / A;
    for (int jb = 0; jb < 4 * ng; jb++) {
        double *md = &m.coef[kCoefHead + kCoefMode * jb];
        md[0] = jb < n_bath ? aj[jb] : 0.0;
        md[1] = jb < n_bath ? bj[jb] + 1.0 : 0.0;
        md[2] = cj[jb];
        md[3] = 0.5 * dt * kk[jb] * aj[jb] / A;
        md[4] = 0.5 * dt * kk[jb] * bj[jb] / A;
        md[5] = w2[jb];
    }
    TRY(g->alloc((void **)&m.coef_dev, 8 * m.coef.size()));
    HIP_TRY(hipMemcpy(m.coef_dev, m.coef.data(), 8 * m.coef.size(), hipMemcpyHostToDevice));
    if (sigma_cells) {
        m.sigma_per_cell = true;
        m.sigma_hash = fnv1a(sigma_cells, 8 * (size_t)mc);
        TRY(g->alloc(&m.sigma_dev, words(mc, g->f64)));
        TRY(write_state(g, m.sigma_dev, mc, sigma_cells));
    }
    for (int lvl = 0; lvl < 2; lvl++)
        for (int c = 0; c < 3; c++) {
            if (!e_active(g->ndim, c)) continue;
            TRY(g->alloc(&m.P[lvl][c], words(mc, g->f64)));
            // the six bath-level arrays are handed out 0, 1, ..., 5 KiB into their allocations (which
            // start on the same large-page boundary): the 512^3 layer's bath launch took 6.26 ms
            // against 6.33 ms with every array at the start of its allocation
            if (ng) TRY(g->alloc(&m.Y[lvl][c], words(mc * 4 * ng, g->f64), 1024 * (size_t)(3 * lvl + c)));
        }
    if (material_id) *material_id = (int)g->mats.size() - 1;
    return FDTDB_OK;
}

// Block of the coefficient table after the modes (layout with the table's): the thermal / anharmonic
// terms, or for a bath stored in 16 bits the coefficients that act on scaled coordinates
static fdtdb_status rebuild_ext(fdtdb_grid_s *g, Material &m) {
    const double dt = g->dt, w02 = m.omega0 * m.omega0;
    const size_t base = kCoefHead + (size_t)kCoefMode * 4 * m.ng;
    double skc = 0.0;
    for (int jb = 0; jb < m.nb; jb++) skc += m.kj[jb] * (m.kj[jb] * dt / (2.0 * (1.0 + 0.5 * m.gj[jb] * dt)));
    const double A = 1.0 + 0.5 * m.gamma0 * dt + 0.5 * dt * skc;
    m.coef.resize(base);
    m.coef[6] = 0.0;
    if (m.bext()) {
        m.coef.resize(base + (size_t)kCoefExt * 4 * m.ng, 0.0);
        if (m.kT > 0.0) m.coef[6] = dt * dt * std::sqrt(2.0 * m.gamma0 * m.kT * w02 / dt) / A;
        for (int jb = 0; jb < m.nb; jb++) {
            const double den = 1.0 + 0.5 * m.gj[jb] * dt;
            double *x = &m.coef[base + (size_t)kCoefExt * jb];
            x[0] = m.kT > 0.0 ? dt * dt * std::sqrt(2.0 * m.gj[jb] * m.kT * w02 / dt) / den : 0.0;
            x[1] = m.lam.empty() ? 0.0 : m.lam[jb] * dt * dt / den;
            x[2] = 0.5 * dt * m.kj[jb] / A;
        }
    } else if (m.yfmt) {
        // per mode, as FP32 (5 floats; the bath recurrence of 16-bit coordinates runs in FP32): a_j, b_j + 1,
        // c_j s, sa_j / s, sb_j / s, packed two to a table word
        const size_t nf = 5 * 4 * (size_t)m.ng;
        m.coef.resize(base + (nf + 1) / 2, 0.0);
        std::vector<float> f(nf + 1, 0.0f);
        for (int jb = 0; jb < 4 * m.ng; jb++) {
            const double *md = &m.coef[kCoefHead + (size_t)kCoefMode * jb];
            float *x = &f[5 * (size_t)jb];
            x[0] = (float)md[0];
            x[1] = (float)md[1];
            x[2] = (float)(md[2] * m.yscale);
            x[3] = (float)(md[3] / m.yscale);
            x[4] = (float)(md[4] / m.yscale);
        }
        std::memcpy(&m.coef[base], f.data(), 4 * nf);
    }
    void *old = m.coef_dev;
    g->release(old);
    m.coef_dev = nullptr;
    TRY(g->alloc((void **)&m.coef_dev, 8 * m.coef.size()));
    HIP_TRY(hipMemcpy(m.coef_dev, m.coef.data(), 8 * m.coef.size(), hipMemcpyHostToDevice));
    return FDTDB_OK;
}

static fdtdb_status ext_target(fdtdb_grid g, int material_id) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "thermal and anharmonic terms are set before the first step");
    if (g->twin || g->orphan) return fail(FDTDB_E_STATE, "thermal and anharmonic baths are not available on Bloch grids");
    if (material_id < 0 || material_id >= (int)g->mats.size() || g->mats[material_id].kind != K_BATH ||
        g->mats[material_id].nb == 0)
        return fail(FDTDB_E_INVALID, "thermal and anharmonic terms apply to a Lorentz-Bath material's bath");
    if (g->mats[material_id].yfmt) return fail(FDTDB_E_STATE, "the bath is stored in 16 bits");
    if (g->mats[material_id].cw_dev) return fail(FDTDB_E_STATE, "the material's bath is replaced by a learned closure");
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_bath_thermal(fdtdb_grid g, int material_id, double kT, uint64_t seed) {
    TRY(ext_target(g, material_id));
    if (!(kT >= 0.0) || !std::isfinite(kT)) return fail(FDTDB_E_INVALID, "kT must be finite and >= 0");
    Material &m = g->mats[material_id];
    m.kT = kT;
    m.seed = seed;
    return rebuild_ext(g, m);
}

fdtdb_status fdtdb_set_bath_anharmonic(fdtdb_grid g, int material_id, const double *lambda, int n) {
    TRY(ext_target(g, material_id));
    Material &m = g->mats[material_id];
    if (n != 0 && (!lambda || n != m.nb)) return fail(FDTDB_E_INVALID, "one quartic coefficient per bath mode (%d)", m.nb);
    for (int jb = 0; jb < n; jb++)
        if (!std::isfinite(lambda[jb])) return fail(FDTDB_E_INVALID, "non-finite quartic coefficient");
    if (n) m.lam.assign(lambda, lambda + n);
    else m.lam.clear();
    return rebuild_ext(g, m);
}

fdtdb_status fdtdb_set_bath_storage(fdtdb_grid g, int material_id, int format, double scale) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "bath storage is chosen before the first step");
    if (g->twin || g->orphan) return fail(FDTDB_E_STATE, "16-bit bath storage is not available on Bloch grids");
    if (material_id < 0 || material_id >= (int)g->mats.size() || g->mats[material_id].kind != K_BATH ||
        g->mats[material_id].nb == 0)
        return fail(FDTDB_E_INVALID, "the storage format applies to a Lorentz-Bath material's bath");
    Material &m = g->mats[material_id];
    if (format < FDTDB_BATH_STATE || format > FDTDB_BATH_BF16) return fail(FDTDB_E_INVALID, "bad storage format");
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(FDTDB_E_INVALID, "scale must be finite and > 0");
    if (m.cw_dev) return fail(FDTDB_E_STATE, "the material's bath is replaced by a learned closure");
    if (m.bext()) return fail(FDTDB_E_STATE, "a thermal or anharmonic bath is kept in the state type");
    if (format != FDTDB_BATH_STATE && (g->ndim != 3 || g->f64 || m.ng != 4))
        return fail(FDTDB_E_INVALID, "16-bit bath storage needs a 3D FP32 grid and 16 bath modes");
    const size_t word = format == FDTDB_BATH_STATE ? g->esize() : 2;
    for (int lvl = 0; lvl < 2; lvl++)
        for (int c = 0; c < 3; c++) {
            if (!m.Y[lvl][c]) continue;
            g->release(m.Y[lvl][c]);
            TRY(g->alloc(&m.Y[lvl][c], (size_t)m.mcells * 4 * m.ng * word, 1024 * (size_t)(3 * lvl + c)));
        }
    m.yfmt = format;
    m.yscale = format == FDTDB_BATH_STATE ? 1.0 : scale;
    return rebuild_ext(g, m);
}

fdtdb_status fdtdb_set_bath_closure(fdtdb_grid g, int material_id, const float *weights, int width,
                                    const double *scales) {
    if (!g || !weights || !scales) return fail(FDTDB_E_INVALID, "null argument");
    if (g->finalized) return fail(FDTDB_E_STATE, "closures must be set before the first step");
    if (g->twin || g->orphan) return fail(FDTDB_E_STATE, "learned closures are not available on Bloch grids");
    if (material_id >= 0 && material_id < (int)g->mats.size() && g->mats[material_id].yfmt)
        return fail(FDTDB_E_STATE, "the closure replaces a bath stored in 16 bits");
    if (material_id >= 0 && material_id < (int)g->mats.size() && g->mats[material_id].bext())
        return fail(FDTDB_E_STATE, "the closure replaces a thermal or anharmonic bath");
    if (material_id < 0 || material_id >= (int)g->mats.size() || g->mats[material_id].kind != K_BATH)
        return fail(FDTDB_E_INVALID, "the closure replaces the bath of a Lorentz-Bath material");
    if (width != kClosureWidth) return fail(FDTDB_E_INVALID, "closure width must be %d", kClosureWidth);
    for (int q = 0; q < 4; q++)
        if (!(scales[q] > 0.0) || !std::isfinite(scales[q])) return fail(FDTDB_E_INVALID, "closure scales must be > 0");
    for (int q = 0; q < kClosureParams; q++)
        if (!std::isfinite(weights[q])) return fail(FDTDB_E_INVALID, "non-finite closure weight");
    Material &m = g->mats[material_id];
    m.weight_hash = fnv1a(weights, sizeof(float) * kClosureParams);
    // the weights, then their transposed copy (layers 1 and 3 of the inference kernel read it)
    if (!m.cw_dev) TRY(g->alloc((void **)&m.cw_dev, 2 * sizeof(float) * kClosureParams));
    std::vector<float> both(2 * (size_t)kClosureParams);
    for (int e = 0; e < kClosureParams; e++) {
        both[e] = weights[e];
        both[kClosureParams + closure_tpos(e)] = weights[e];
    }
    HIP_TRY(hipMemcpy(m.cw_dev, both.data(), 2 * sizeof(float) * kClosureParams, hipMemcpyHostToDevice));
    for (int c = 0; c < 3; c++)
        if (e_active(g->ndim, c) && !m.hid[c]) TRY(g->alloc(&m.hid[c], 16 * (size_t)m.mcells));
    m.cscale[0] = scales[0];
    m.cscale[1] = scales[1];
    m.cscale[2] = scales[2];
    m.cscale[3] = 1.0 / scales[3];
    for (int lvl = 0; lvl < 2; lvl++)          // the explicit bath coordinates are no longer used
        for (int c = 0; c < 3; c++) g->release(m.Y[lvl][c]);
    m.kind = K_CLOSURE;
    return FDTDB_OK;
}

fdtdb_status fdtdb_get_closure_state(fdtdb_grid g, int material_id, int component, double *out) {
    if (!g || !out || material_id < 0 || material_id >= (int)g->mats.size() || component < 0 || component > 2)
        return fail(FDTDB_E_INVALID, "bad argument");
    Material &m = g->mats[material_id];
    if (m.kind != K_CLOSURE || !m.hid[component]) return fail(FDTDB_E_INVALID, "no closure state");
    TRY(sync(g));
    std::vector<float> tmp(4 * (size_t)m.mcells);
    HIP_TRY(hipMemcpy(tmp.data(), m.hid[component], 16 * (size_t)m.mcells, hipMemcpyDeviceToHost));
    for (size_t q = 0; q < tmp.size(); q++) out[q] = tmp[q];
    return FDTDB_OK;
}

fdtdb_status fdtdb_bath_params(int form, double omega0, double gamma0, int n_bath, double width, double bath_gamma,
                               double dephasing, double *omega_j, double *gamma_j, double *k_j) {
    if (n_bath < 2 || !omega_j || !gamma_j || !k_j || form < 0 || form > 2 || !(width > 0.0))
        return fail(FDTDB_E_INVALID, "bath_params: need n_bath >= 2, width > 0, form in {0,1,2}");
    const double dw = width / (n_bath - 1);
    const double kb = std::sqrt(2.0 * dw / M_PI * dephasing);
    const double G = gamma0 + dephasing;
    for (int jb = 0; jb < n_bath; jb++) {
        const double w = omega0 - width / 2 + width * jb / (n_bath - 1);
        omega_j[jb] = w;
        gamma_j[jb] = bath_gamma;
        const double d = w - omega0;
        if (form == 0) k_j[jb] = kb;
        else if (form == 1) k_j[jb] = kb * std::sqrt(G * G / (G * G + d * d));
        else k_j[jb] = kb * std::exp(-d * d / (4.0 * G * G));
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_add_source(fdtdb_grid g, int component, const fdtdb_box *box, double omega_c, double width,
                              double amplitude, const double *profile, int *source_id) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "sources must be added before the first step");
    if (!box_ok(g, box)) return fail(FDTDB_E_INVALID, "source box outside the grid");
    if (component < 0 || component > 2 || !e_active(g->ndim, component))
        return fail(FDTDB_E_INVALID, "source component not carried by a %dD grid", g->ndim);
    if (!(width > 0.0)) return fail(FDTDB_E_INVALID, "width must be > 0");
    if ((int)g->srcs.size() >= kMaxSources) return fail(FDTDB_E_INVALID, "at most %d sources", kMaxSources);
    // the box must sit in one eps_inf
    double eps = -1.0;
    for (int64_t i = box->lo[0]; i < box->hi[0]; i++)
        for (int64_t j = box->lo[1]; j < box->hi[1]; j++)
            for (int64_t k = box->lo[2]; k < box->hi[2]; k++) {
                double e = 1.0;
                for (auto &m : g->mats)
                    if (i >= m.lo[0] && i < m.hi[0] && j >= m.lo[1] && j < m.hi[1] && k >= m.lo[2] && k < m.hi[2]) e = m.eps;
                if (eps < 0) eps = e;
                else if (e != eps) return fail(FDTDB_E_INVALID, "source box spans several eps_inf values");
            }
    Source s;
    s.comp = component;
    for (int a = 0; a < 3; a++) { s.lo[a] = box->lo[a]; s.hi[a] = box->hi[a]; }
    s.omega_c = omega_c;
    s.width = width;
    s.amplitude = amplitude;
    s.eps = eps;
    if (profile) {
        long long nc = 1;
        for (int a = 0; a < 3; a++) nc *= box->hi[a] - box->lo[a];
        s.profile.assign(profile, profile + nc);
    }
    g->srcs.push_back(std::move(s));
    if (source_id) *source_id = (int)g->srcs.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_add_dft_flux(fdtdb_grid g, int axis, const fdtdb_box *plane, int nfreq, const double *omega,
                                int *monitor_id) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "monitors must be added before the first step");
    if (axis < 0 || axis >= g->ndim) return fail(FDTDB_E_INVALID, "bad axis");
    if (!box_ok(g, plane) || plane->hi[axis] != plane->lo[axis] + 1)
        return fail(FDTDB_E_INVALID, "flux plane must be inside the grid and one cell thick along its axis");
    if (g->twin && g->bph[axis] != 0.0 && plane->lo[axis] == 0)
        return fail(FDTDB_E_INVALID, "a flux plane normal to a Bloch axis cannot sit at its first cell");
    if (nfreq < 1 || !omega) return fail(FDTDB_E_INVALID, "need frequencies");
    Dft d;
    d.axis = axis;
    d.npts = 1;
    for (int a = 0; a < 3; a++) {
        d.lo[a] = plane->lo[a];
        d.hi[a] = plane->hi[a];
        d.npts *= (int)(plane->hi[a] - plane->lo[a]);
    }
    d.nf = nfreq;
    d.t1 = curl_a1(axis);
    d.t2 = curl_a2(axis);
    d.omega.assign(omega, omega + nfreq);
    TRY(g->alloc((void **)&d.omega_dev, 8 * (size_t)nfreq));
    HIP_TRY(hipMemcpy(d.omega_dev, omega, 8 * (size_t)nfreq, hipMemcpyHostToDevice));
    TRY(g->alloc((void **)&d.stage, 8 * (size_t)kDftSlots * 4 * d.npts));
    TRY(g->alloc((void **)&d.tw, 32 * (size_t)kDftSlots * nfreq));
    TRY(g->alloc((void **)&d.acc, 16 * (size_t)4 * nfreq * d.npts));
    TRY(g->alloc((void **)&d.flux_dev, 8 * (size_t)nfreq));
    g->dfts.push_back(std::move(d));
    if (monitor_id) *monitor_id = (int)g->dfts.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_add_energy_monitor(fdtdb_grid g, const fdtdb_box *box, int every, int *monitor_id) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (g->finalized) return fail(FDTDB_E_STATE, "monitors must be added before the first step");
    if (!box_ok(g, box) || every < 1) return fail(FDTDB_E_INVALID, "bad energy box or period");
    if (in_pml(g, box->lo, box->hi)) return fail(FDTDB_E_INVALID, "energy box overlaps the CPML layer");
    if ((int)g->ens.size() >= kMaxEnergy) return fail(FDTDB_E_INVALID, "at most %d energy monitors", kMaxEnergy);
    Energy e;
    for (int a = 0; a < 3; a++) { e.lo[a] = box->lo[a]; e.hi[a] = box->hi[a]; }
    e.every = every;
    g->ens.push_back(e);
    if (monitor_id) *monitor_id = (int)g->ens.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_add_probe(fdtdb_grid g, int material_id, int component, int n, const int64_t *cells,
                             int64_t nsteps, int *probe_id) {
    if (!g || !cells) return fail(FDTDB_E_INVALID, "null argument");
    if (g->finalized) return fail(FDTDB_E_STATE, "probes must be added before the first step");
    if (material_id < 0 || material_id >= (int)g->mats.size()) return fail(FDTDB_E_INVALID, "bad material");
    Material &mt = g->mats[material_id];
    if (mt.kind != K_BATH && mt.kind != K_CLOSURE) return fail(FDTDB_E_INVALID, "probes record Lorentz-Bath cells");
    if (component < 0 || component > 2 || !e_active(g->ndim, component)) return fail(FDTDB_E_INVALID, "bad component");
    if (n < 1 || nsteps < 1) return fail(FDTDB_E_INVALID, "need n >= 1 cells and nsteps >= 1");
    Probe p;
    p.mat = material_id;
    p.comp = component;
    p.n = n;
    p.capacity = nsteps;
    std::vector<int> q(n), m(n);
    for (int i = 0; i < n; i++) {
        if (cells[i] < 0 || cells[i] >= mt.mcells) return fail(FDTDB_E_INVALID, "probe cell %d outside the material", i);
        const long long c = cells[i];
        const long long ii = c / ((long long)mt.mext[1] * mt.mext[2]);
        const long long rem = c - ii * mt.mext[1] * mt.mext[2];
        const long long jj = rem / mt.mext[2], kk = rem - jj * mt.mext[2];
        q[i] = (int)(((mt.lo[0] + ii) * g->n[1] + (mt.lo[1] + jj)) * g->n[2] + (mt.lo[2] + kk));
        m[i] = (int)c;
    }
    TRY(g->alloc((void **)&p.q, 4 * (size_t)n));
    TRY(g->alloc((void **)&p.m, 4 * (size_t)n));
    TRY(g->alloc((void **)&p.E, 4 * (size_t)n * (size_t)nsteps));
    TRY(g->alloc((void **)&p.P, 4 * (size_t)n * (size_t)nsteps));
    HIP_TRY(hipMemcpy(p.q, q.data(), 4 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p.m, m.data(), 4 * (size_t)n, hipMemcpyHostToDevice));
    g->probes.push_back(p);
    if (probe_id) *probe_id = (int)g->probes.size() - 1;
    return FDTDB_OK;
}

fdtdb_status fdtdb_probe_data(fdtdb_grid g, int probe_id, float *E, float *P, int to_device) {
    if (!g || !E || !P || probe_id < 0 || probe_id >= (int)g->probes.size()) return fail(FDTDB_E_INVALID, "bad argument");
    TRY(sync(g));
    const Probe &p = g->probes[probe_id];
    const size_t bytes = 4 * (size_t)p.n * (size_t)p.capacity;
    const hipMemcpyKind k = to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (to_device) HIP_TRY(hipDeviceSynchronize());   // work another stream has pending on E, P finishes first
    HIP_TRY(hipMemcpy(E, p.E, bytes, k));
    HIP_TRY(hipMemcpy(P, p.P, bytes, k));
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_graph(fdtdb_grid g, int chunk_steps) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (chunk_steps < 0) return fail(FDTDB_E_INVALID, "chunk must be >= 0");
    if (g->graph) { (void)hipGraphExecDestroy(g->graph); g->graph = nullptr; }
    int c = chunk_steps;
    if (c > 0) {
        if (!g->dfts.empty()) c = ((c + kDftSlots - 1) / kDftSlots) * kDftSlots;
        c += c & 1;
    }
    g->graph_chunk = c;
    return FDTDB_OK;
}

fdtdb_status fdtdb_step(fdtdb_grid g, int64_t nsteps) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (nsteps < 0) return fail(FDTDB_E_INVALID, "nsteps < 0");
    if (g->orphan) return fail(FDTDB_E_STATE, "the other part of this Bloch grid was destroyed");
    if (g->twin) {
        if (g->part != 0) return fail(FDTDB_E_STATE, "a Bloch pair steps through its real part");
        fdtdb_grid_s *im = g->twin;
        if (g->dfts.size() != im->dfts.size()) return fail(FDTDB_E_STATE, "the parts need the same flux monitors");
        for (size_t i = 0; i < g->dfts.size(); i++)
            if (g->dfts[i].npts != im->dfts[i].npts || g->dfts[i].nf != im->dfts[i].nf)
                return fail(FDTDB_E_STATE, "the parts need the same flux monitors");
        TRY(finalize(g));
        TRY(finalize(im));
        if (g->steps != im->steps) return fail(FDTDB_E_STATE, "the two parts of the Bloch pair are at different steps");
        TRY(ensure_energy_capacity(g, g->steps + nsteps));
        TRY(ensure_energy_capacity(im, im->steps + nsteps));
        for (int64_t s = 0; s < nsteps; s++) TRY(enqueue_pair_step(g));
        return FDTDB_OK;
    }
    TRY(finalize(g));
    TRY(ensure_energy_capacity(g, g->steps + nsteps));
    int64_t left = nsteps;
    while (left > 0) {
        bool aligned = true;
        for (auto &d : g->dfts) aligned = aligned && d.nstaged == 0;
        const int chunk = g->graph_chunk;
        if (chunk > 0 && !g->profiling && left >= chunk && aligned && (g->steps & 1) == 0) {
            if (!g->graph) {
                hipGraph_t graph;
                HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
                const long long s0 = g->steps;
                fdtdb_status st = FDTDB_OK;
                for (int s = 0; s < chunk && st == FDTDB_OK; s++) st = enqueue_step(g);
                hipError_t ce = hipStreamEndCapture(g->stream, &graph);
                g->steps = s0;   // the captured steps run below, at replay
                if (st != FDTDB_OK) return st;
                if (ce != hipSuccess) return fail(FDTDB_E_DEVICE, "graph capture: %s", hipGetErrorString(ce));
                HIP_TRY(hipGraphInstantiate(&g->graph, graph, nullptr, nullptr, 0));
                (void)hipGraphDestroy(graph);
            }
            HIP_TRY(hipGraphLaunch(g->graph, g->stream));
            g->steps += chunk;
            left -= chunk;
        } else {
            TRY(enqueue_step(g));
            left -= 1;
        }
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_pair_bloch(fdtdb_grid re, fdtdb_grid im, const double *phase) {
    if (!re || !im || !phase || re == im) return fail(FDTDB_E_INVALID, "need two grids and the phases");
    if (re->finalized || im->finalized) return fail(FDTDB_E_STATE, "grids are paired before their first step");
    if (re->twin || im->twin || re->orphan || im->orphan) return fail(FDTDB_E_STATE, "grid already paired");
    if (re->ndim != im->ndim || re->f64 != im->f64 || re->dt != im->dt || re->R0 != im->R0)
        return fail(FDTDB_E_INVALID, "the parts need the same dimension, precision and time step");
    // one stream for both parts: an imaginary part that created its own stream takes the real part's
    if (re->stream != im->stream && !im->own_stream)
        return fail(FDTDB_E_INVALID, "the parts need the same stream");
    for (int a = 0; a < 3; a++) {
        if (re->n[a] != im->n[a] || re->bc[a] != im->bc[a] || re->pml[a] != im->pml[a])
            return fail(FDTDB_E_INVALID, "the parts need the same shape and boundaries");
        if (!std::isfinite(phase[a])) return fail(FDTDB_E_INVALID, "non-finite phase");
        if (phase[a] != 0.0 && (a >= re->ndim || re->bc[a] != FDTDB_BC_PERIODIC))
            return fail(FDTDB_E_INVALID, "a Bloch phase needs a periodic axis of the grid");
    }
    for (const fdtdb_grid_s *g : {re, im})
        for (auto &m : g->mats) {
            if (m.cw_dev) return fail(FDTDB_E_STATE, "learned closures are not available on Bloch grids");
            if (m.yfmt) return fail(FDTDB_E_STATE, "16-bit bath storage is not available on Bloch grids");
            if (m.bext()) return fail(FDTDB_E_STATE, "thermal and anharmonic baths are not available on Bloch grids");
        }
    if (re->dfts.size() != im->dfts.size()) return fail(FDTDB_E_INVALID, "the parts need the same flux monitors");
    for (size_t i = 0; i < re->dfts.size(); i++) {
        const Dft &a = re->dfts[i], &b = im->dfts[i];
        if (a.axis != b.axis || a.npts != b.npts || a.nf != b.nf)
            return fail(FDTDB_E_INVALID, "the parts need the same flux monitors");
        if (phase[a.axis] != 0.0 && a.lo[a.axis] == 0)
            return fail(FDTDB_E_INVALID, "a flux plane normal to a Bloch axis cannot sit at its first cell");
    }
    if (re->stream != im->stream) {
        HIP_TRY(hipStreamSynchronize(im->stream));
        HIP_TRY(hipStreamDestroy(im->stream));
        im->stream = re->stream;
        im->own_stream = false;
    }
    re->twin = im;
    im->twin = re;
    re->part = 0;
    im->part = 1;
    for (int a = 0; a < 3; a++) re->bph[a] = im->bph[a] = phase[a];
    return FDTDB_OK;
}

fdtdb_status fdtdb_steps_done(fdtdb_grid g, int64_t *steps) {
    if (!g || !steps) return fail(FDTDB_E_INVALID, "null argument");
    *steps = g->steps;
    return FDTDB_OK;
}

// Energy watchdog: once every source has ended (t > 2 t0 of each), a passive grid's exact discrete
// energy cannot grow (eq:H_full with the damping of eq:EOM_LorentzBath and the absorbing layers only
// take energy out; what the layers hand back is their reflection, orders of magnitude below), so a
// monitor over every cell outside the CPML layers whose total exceeds twice its smallest value since
// then, while above 1 % of its value when the sources ended, marks an instability long before any
// field overflows.
fdtdb_status energy_watchdog(fdtdb_grid_s *g) {
    if (g->twin || g->orphan) return FDTDB_OK;   // a Bloch pair conserves the sum over both parts only
    for (auto &m : g->mats)                      // a thermal bath feeds energy in: the grid is not passive
        if (m.kT > 0.0) return FDTDB_OK;
    double t_off = 0.0;
    for (auto &x : g->srcs) t_off = std::max(t_off, 10.0 / x.width);
    for (auto &e : g->ens) {
        bool whole = true;
        for (int a = 0; a < 3; a++) {
            const int64_t l = g->bc[a] == FDTDB_BC_PML ? g->pml[a] : 0;
            whole &= e.lo[a] <= l && e.hi[a] >= g->n[a] - l;
        }
        if (!whole) continue;
        const long long n = g->steps == 0 ? 0 : (g->steps - 1) / e.every + 1;
        const long long m = std::min<long long>(n, e.capacity);
        if (m <= e.checked) continue;
        std::vector<double> v(3 * (size_t)(m - e.checked));
        HIP_TRY(hipMemcpy(v.data(), e.out + 3 * e.checked, 8 * v.size(), hipMemcpyDeviceToHost));
        for (long long k = e.checked; k < m; k++) {
            const double *x = &v[3 * (size_t)(k - e.checked)];
            const double tot = x[0] + x[1] + x[2];
            if ((double)(k * e.every) * g->dt <= t_off) continue;
            if (e.ref < 0.0) {
                e.ref = tot;
                e.low = tot;
                continue;
            }
            e.low = std::min(e.low, tot);
            if (tot > 2.0 * e.low && tot > 1e-2 * e.ref)
                return fail(FDTDB_E_DIVERGED, "energy of a whole-grid monitor grew from %.6g to %.6g after the sources "
                                              "ended (sample at step %lld)", e.low, tot, k * e.every);
        }
        e.checked = m;
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_synchronize(fdtdb_grid g) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    HIP_TRY(hipMemsetAsync(g->flag_dev, 0, sizeof(int), g->stream));
    for (int c = 0; c < 3; c++) {
        if (g->E[c]) HIP_TRY(launch_nonfinite(g->f64, g->E[c], g->ncell, g->flag_dev, g->stream));
        if (g->H[c]) HIP_TRY(launch_nonfinite(g->f64, g->H[c], g->ncell, g->flag_dev, g->stream));
    }
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, g->flag_dev, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    if (flag) return fail(FDTDB_E_DIVERGED, "non-finite field after %lld steps", (long long)g->steps);
    return energy_watchdog(g);
}

fdtdb_status fdtdb_dft_flux(fdtdb_grid g, int id, double *flux, double *raw) {
    if (!g || id < 0 || id >= (int)g->dfts.size() || (!flux && !raw)) return fail(FDTDB_E_INVALID, "bad monitor");
    if (flux && g->twin && g->part != 0) return fail(FDTDB_E_STATE, "the flux of a Bloch pair is read from its real part");
    if (flux && !g->twin && g->orphan) return fail(FDTDB_E_STATE, "the other part of this Bloch grid was destroyed");
    Dft &d = g->dfts[id];
    if (flux && g->twin && id >= (int)g->twin->dfts.size()) return fail(FDTDB_E_STATE, "monitor missing on the other part");
    Dft *di = g->twin && flux ? &g->twin->dfts[id] : nullptr;
    if (g->finalized) TRY(flush_dft(g, d));
    if (di && g->twin->finalized) TRY(flush_dft(g->twin, *di));
    if (flux) {
        if (g->finalized) HIP_TRY(launch_dft_flux(d.acc, di ? di->acc : nullptr, d.npts, d.nf, d.flux_dev, g->stream));
        TRY(sync(g));
        HIP_TRY(hipMemcpy(flux, d.flux_dev, 8 * (size_t)d.nf, hipMemcpyDeviceToHost));
    } else {
        TRY(sync(g));
    }
    if (raw) {
        // device layout [field][f][p] -> ABI layout [field][p][f]
        std::vector<double2> tmp((size_t)4 * d.nf * d.npts);
        HIP_TRY(hipMemcpy(tmp.data(), d.acc, 16 * tmp.size(), hipMemcpyDeviceToHost));
        for (int fld = 0; fld < 4; fld++)
            for (int f = 0; f < d.nf; f++)
                for (int p = 0; p < d.npts; p++) {
                    const double2 v = tmp[((size_t)fld * d.nf + f) * d.npts + p];
                    double *o = raw + (((size_t)fld * d.npts + p) * d.nf + f) * 2;
                    o[0] = v.x;
                    o[1] = v.y;
                }
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_energy(fdtdb_grid g, int id, double *out, int64_t capacity, int64_t *n_samples) {
    if (!g || id < 0 || id >= (int)g->ens.size()) return fail(FDTDB_E_INVALID, "bad monitor");
    Energy &e = g->ens[id];
    TRY(sync(g));
    const long long n = g->steps == 0 ? 0 : (g->steps - 1) / e.every + 1;
    if (n_samples) *n_samples = n;
    const long long m = std::min<long long>(n, capacity);
    if (out && m > 0) HIP_TRY(hipMemcpy(out, e.out, 24 * (size_t)m, hipMemcpyDeviceToHost));
    return FDTDB_OK;
}

fdtdb_status fdtdb_get_field(fdtdb_grid g, int component, void *dst, int dst_is_device) {
    if (!g || !dst || component < 0 || component > 5) return fail(FDTDB_E_INVALID, "bad component");
    TRY(sync(g));
    const void *src = component < 3 ? g->E[component] : g->H[component - 3];
    if (!dst_is_device) return read_state(g, src, g->ncell, static_cast<double *>(dst));
    // the destination may still have work pending on another stream (a caller's fill of a fresh buffer):
    // wait for the whole device, so that this copy is the last write
    HIP_TRY(hipDeviceSynchronize());
    double *out = static_cast<double *>(dst);
    if (!src) HIP_TRY(hipMemsetAsync(out, 0, 8 * (size_t)g->ncell, g->stream));
    else if (g->f64) HIP_TRY(hipMemcpyAsync(out, src, 8 * (size_t)g->ncell, hipMemcpyDeviceToDevice, g->stream));
    else HIP_TRY(launch_to_f64(false, src, g->ncell, out, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_field(fdtdb_grid g, int component, const double *in) {
    if (!g || !in || component < 0 || component > 5) return fail(FDTDB_E_INVALID, "bad component");
    void *dst = component < 3 ? g->E[component] : g->H[component - 3];
    if (!dst) return fail(FDTDB_E_INVALID, "component not carried by this grid");
    TRY(sync(g));
    return write_state(g, dst, g->ncell, in);
}

fdtdb_status fdtdb_get_polarization(fdtdb_grid g, int mid, int c, int level, double *out) {
    if (!g || mid < 0 || mid >= (int)g->mats.size() || c < 0 || c > 2 || level < 0 || level > 1 || !out)
        return fail(FDTDB_E_INVALID, "bad argument");
    Material &m = g->mats[mid];
    if (m.kind == K_BACKGROUND || !e_active(g->ndim, c)) return fail(FDTDB_E_INVALID, "no polarization");
    TRY(sync(g));
    if (m.kind == K_DRUDE) {
        if (level == 1) {
            std::fill(out, out + m.mcells, 0.0);
            return FDTDB_OK;
        }
        return read_state(g, m.P[0][c], m.mcells, out);
    }
    const int slot = (int)((g->steps + level) & 1);
    if (m.kind == K_MULTI) {     // the total polarization: the sum of the terms (Lorentz terms only)
        for (int p = 0; p < m.nterm; p++)
            if (m.coef[kCoefHead + kCoefMode * p + 5] != 0.0)
                return fail(FDTDB_E_INVALID, "a Drude term stores its increment only: read the terms one by one");
        std::vector<double> t((size_t)m.mcells);
        std::fill(out, out + m.mcells, 0.0);
        for (int p = 0; p < m.nterm; p++) {
            TRY(read_state(g, static_cast<char *>(m.P[slot][c]) + (size_t)p * m.mcells * (g->f64 ? 8 : 4), m.mcells,
                           t.data()));
            for (long long q = 0; q < m.mcells; q++) out[q] += t[q];
        }
        return FDTDB_OK;
    }
    return read_state(g, m.P[slot][c], m.mcells, out);
}

fdtdb_status fdtdb_get_polarization_term(fdtdb_grid g, int mid, int c, int level, int term, double *out) {
    if (!g || mid < 0 || mid >= (int)g->mats.size() || c < 0 || c > 2 || level < 0 || level > 1 || !out)
        return fail(FDTDB_E_INVALID, "bad argument");
    Material &m = g->mats[mid];
    if (m.kind != K_MULTI || term < 0 || term >= m.nterm || !e_active(g->ndim, c))
        return fail(FDTDB_E_INVALID, "no such term");
    TRY(sync(g));
    if (m.coef[kCoefHead + kCoefMode * term + 5] != 0.0) {      // Drude term: its increment, in the level-0 slot
        if (level == 1) {
            std::fill(out, out + m.mcells, 0.0);
            return FDTDB_OK;
        }
        return read_state(g, static_cast<char *>(m.P[(int)(g->steps & 1)][c]) + (size_t)term * m.mcells * (g->f64 ? 8 : 4),
                          m.mcells, out);
    }
    const int slot = (int)((g->steps + level) & 1);
    return read_state(g, static_cast<char *>(m.P[slot][c]) + (size_t)term * m.mcells * (g->f64 ? 8 : 4), m.mcells, out);
}

fdtdb_status fdtdb_get_bath(fdtdb_grid g, int mid, int c, int level, double *out) {
    if (!g || mid < 0 || mid >= (int)g->mats.size() || c < 0 || c > 2 || level < 0 || level > 1 || !out)
        return fail(FDTDB_E_INVALID, "bad argument");
    Material &m = g->mats[mid];
    if (m.kind != K_BATH || m.nb == 0 || !e_active(g->ndim, c)) return fail(FDTDB_E_INVALID, "no bath");
    TRY(sync(g));
    const int slot = (int)((g->steps + level) & 1);
    std::vector<double> tmp((size_t)m.mcells * 4 * m.ng);
    if (m.yfmt) {   // 16-bit storage: widened on the device, scale removed
        double *d = nullptr;
        TRY(g->alloc((void **)&d, 8 * tmp.size()));
        hipError_t e = launch_bath16_to_f64(m.Y[slot][c], (long long)tmp.size(), m.yfmt, 1.0 / m.yscale, d, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e == hipSuccess) e = hipMemcpy(tmp.data(), d, 8 * tmp.size(), hipMemcpyDeviceToHost);
        void *dv = d;
        g->release(dv);
        if (e != hipSuccess) return fail(FDTDB_E_DEVICE, "bath read-out: %s", hipGetErrorString(e));
    } else {
        TRY(read_state(g, m.Y[slot][c], (long long)tmp.size(), tmp.data()));
    }
    // device layout [group][cell][4] (16-bit storage: [word][cell][8]) -> [mode][cell]
    const int per = m.yfmt ? 8 : 4;
    for (int jb = 0; jb < m.nb; jb++)
        for (long long q = 0; q < m.mcells; q++)
            out[(size_t)jb * m.mcells + q] = tmp[((size_t)(jb / per) * m.mcells + q) * per + (jb % per)];
    return FDTDB_OK;
}


fdtdb_status fdtdb_save_state(fdtdb_grid g, const char *path) {
    if (!g || !path) return fail(FDTDB_E_INVALID, "null argument");
    TRY(finalize(g));
    std::vector<std::pair<void *, size_t>> bufs;
    TRY(state_buffers(g, g->steps, bufs));
    HIP_TRY(hipStreamSynchronize(g->stream));
    File fl;
    fl.f = fopen(path, "wb");
    if (!fl.f) return fail(FDTDB_E_INVALID, "cannot open %s for writing", path);
    const uint64_t fp = fingerprint(g);
    const int64_t steps = g->steps;
    const int32_t nbuf = (int32_t)bufs.size(), ndft = (int32_t)g->dfts.size();
    bool ok = fwrite(kStateMagic, 1, 8, fl.f) == 8 && fwrite(&fp, 8, 1, fl.f) == 1 && fwrite(&steps, 8, 1, fl.f) == 1 &&
              fwrite(&nbuf, 4, 1, fl.f) == 1 && fwrite(&ndft, 4, 1, fl.f) == 1;
    for (auto &d : g->dfts) {
        const int32_t ns = d.nstaged;
        ok = ok && fwrite(&ns, 4, 1, fl.f) == 1;
    }
    std::vector<char> host;
    for (auto &b : bufs) {
        if (!ok) break;
        const uint64_t nb = b.second;
        host.resize(nb);
        HIP_TRY(hipMemcpy(host.data(), b.first, nb, hipMemcpyDeviceToHost));
        ok = fwrite(&nb, 8, 1, fl.f) == 1 && fwrite(host.data(), 1, nb, fl.f) == nb;
    }
    if (!ok) return fail(FDTDB_E_INVALID, "write to %s failed", path);
    if (fclose(fl.f) != 0) { fl.f = nullptr; return fail(FDTDB_E_INVALID, "closing %s failed", path); }
    fl.f = nullptr;
    return FDTDB_OK;
}

fdtdb_status fdtdb_load_state(fdtdb_grid g, const char *path) {
    if (!g || !path) return fail(FDTDB_E_INVALID, "null argument");
    TRY(finalize(g));
    File fl;
    fl.f = fopen(path, "rb");
    if (!fl.f) return fail(FDTDB_E_INVALID, "cannot open %s", path);
    char magic[8];
    uint64_t fp = 0;
    int64_t steps = 0;
    int32_t nbuf = 0, ndft = 0;
    if (fread(magic, 1, 8, fl.f) != 8 || memcmp(magic, kStateMagic, 8) != 0)
        return fail(FDTDB_E_STATE, "%s is not a grid state file", path);
    if (fread(&fp, 8, 1, fl.f) != 1 || fread(&steps, 8, 1, fl.f) != 1 || fread(&nbuf, 4, 1, fl.f) != 1 ||
        fread(&ndft, 4, 1, fl.f) != 1 || steps < 0)
        return fail(FDTDB_E_STATE, "truncated header in %s", path);
    if (fp != fingerprint(g) || ndft != (int32_t)g->dfts.size())
        return fail(FDTDB_E_STATE, "%s was written by a grid with another set-up", path);
    std::vector<int32_t> staged(ndft);
    for (auto &ns : staged)
        if (fread(&ns, 4, 1, fl.f) != 1 || ns < 0 || ns >= kDftSlots) return fail(FDTDB_E_STATE, "bad header in %s", path);
    TRY(ensure_energy_capacity(g, steps));
    std::vector<std::pair<void *, size_t>> bufs;
    TRY(state_buffers(g, steps, bufs));
    if ((size_t)nbuf != bufs.size()) return fail(FDTDB_E_STATE, "%s holds %d buffers, the grid %zu", path, nbuf, bufs.size());
    HIP_TRY(hipStreamSynchronize(g->stream));
    // read everything before touching the device, so that a short file leaves the grid unchanged
    std::vector<std::vector<char>> host(bufs.size());
    for (size_t i = 0; i < bufs.size(); i++) {
        uint64_t nb = 0;
        if (fread(&nb, 8, 1, fl.f) != 1 || nb != bufs[i].second)
            return fail(FDTDB_E_STATE, "buffer %zu of %s has the wrong size", i, path);
        host[i].resize(nb);
        if (fread(host[i].data(), 1, nb, fl.f) != nb) return fail(FDTDB_E_STATE, "truncated buffer %zu in %s", i, path);
    }
    for (size_t i = 0; i < bufs.size(); i++)
        HIP_TRY(hipMemcpy(bufs[i].first, host[i].data(), bufs[i].second, hipMemcpyHostToDevice));
    g->steps = steps;
    for (size_t i = 0; i < g->dfts.size(); i++) g->dfts[i].nstaged = staged[i];
    for (auto &e : g->ens) {          // the watchdog re-reads the restored samples from the start
        e.checked = 0;
        e.ref = -1.0;
        e.low = 0.0;
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_get_stats(fdtdb_grid g, fdtdb_stats *out) {
    if (!g || !out) return fail(FDTDB_E_INVALID, "null argument");
    TRY(finalize(g));
    fdtdb_stats s{};
    s.cells = g->ncell;
    double be = 0.0, bh = 0.0;
    for (auto &r : g->hregions) {
        double e, h;
        region_bytes(g, r, &e, &h);
        bh += h * (double)r.cells();
    }
    for (auto &r : g->regions) {
        double e, h;
        region_bytes(g, r, &e, &h);
        be += e * (double)r.cells();
        if (r.mat >= 0 && g->mats[r.mat].kind != K_BACKGROUND) {
            s.dispersive_cells += r.cells();
            if (g->mats[r.mat].nb && g->mats[r.mat].kind == K_BATH) s.bath_cells += r.cells();
        }
    }
    s.bytes_per_step_e = be;
    s.bytes_per_step_h = bh;
    s.bytes_per_step = be + bh;
    s.launches_per_step = g->launches_per_step;
    *out = s;
    return FDTDB_OK;
}

fdtdb_status fdtdb_set_profiling(fdtdb_grid g, int on) {
    if (!g) return fail(FDTDB_E_INVALID, "null grid");
    if (on < 0 || on > 2) return fail(FDTDB_E_INVALID, "profiling mode must be 0, 1 or 2");
    g->profiling = on;
    return FDTDB_OK;
}

fdtdb_status fdtdb_kernel_records(fdtdb_grid g, fdtdb_kernel_record *out, int capacity, int *count) {
    if (!g || !count) return fail(FDTDB_E_INVALID, "null argument");
    TRY(finalize(g));
    TRY(collect_events(g));
    *count = (int)g->records.size();
    if (out)
        for (int i = 0; i < std::min(capacity, (int)g->records.size()); i++) out[i] = g->records[i];
    return FDTDB_OK;
}

}  // extern "C"
