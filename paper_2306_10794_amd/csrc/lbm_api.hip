// lbm_api.hip -- the C ABI: parameter validation, workspace carving, context
// life cycle, and the ordering of the kernel launches on the caller's stream.
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_internal.hpp"

using namespace lbm;

namespace {

thread_local std::string g_create_err;

constexpr size_t ALIGN = 256;

size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

std::string check_params(const lbm_params &p) {
    char b[256];
    if (p.dim != 2 && p.dim != 3) return "dim must be 2 or 3";
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return "nx, ny, nz must be >= 1";
    if (p.dim == 2 && (p.nz != 1 || p.fluid_q != 9)) return "dim = 2 requires nz = 1 and fluid_q = 9";
    if (p.dim == 3 && p.fluid_q != 19) return "dim = 3 requires fluid_q = 19";
    if (p.dim == 3 && p.nz < 2) return "dim = 3 requires nz >= 2";
    if (!(p.solute_q == p.fluid_q || (p.fluid_q == 9 && p.solute_q == 5) || (p.fluid_q == 19 && p.solute_q == 7)))
        return "solute_q must equal fluid_q, or be 5 (D2Q5) with D2Q9 or 7 (D3Q7) with D3Q19";
    if (p.precision != LBM_FP64 && p.precision != LBM_FP32_DEV) return "unknown precision";
    if (p.rbc_mechanics != LBM_PRECOLL && p.rbc_mechanics != LBM_POSTCOLL) return "unknown rbc_mechanics";
    if (p.rbc_scheme < LBM_SNEW || p.rbc_scheme > LBM_ABB) return "unknown rbc_scheme";
    if (!(p.tau_ns > 0.5) || !(p.tau_ad > 0.5)) return "tau_ns and tau_ad must be > 1/2";
    if (!(p.j0 < 1.0)) return "j0 must be < 1 (negative selects the standard weights)";
    if (!(p.v_m >= 0.0) || !(p.a_m >= 0.0)) return "v_m and a_m must be >= 0";
    if (!(p.k_r >= 0.0)) return "k_r must be >= 0";
    for (int d = 0; d < 3; d++)
        if (p.periodic[d] != 0 && p.periodic[d] != 1) return "periodic[] entries must be 0 or 1";
    if (p.xwrap_shift_y != 0) {
        if (!p.periodic[0] || !p.periodic[1]) return "xwrap_shift_y needs periodic x and y";
        if (p.xwrap_shift_y <= -p.ny || p.xwrap_shift_y >= p.ny) return "|xwrap_shift_y| must be < ny";
    }
    if (p.inlet_axis < -1 || p.inlet_axis >= p.dim) return "inlet_axis must be -1 or an axis of the lattice";
    if (p.inlet_axis >= 0 && p.xwrap_shift_y != 0) return "an inlet axis is incompatible with xwrap_shift_y";
    const double N = (double)p.nx * p.ny * p.nz;
    if (N >= 2147483647.0) {
        snprintf(b, sizeof b, "lattice of %.0f nodes exceeds 2^31 - 1", N);
        return b;
    }
    if (p.phase_change != 0 && p.phase_change != 1) return "phase_change must be 0 or 1";
    if (p.collision != LBM_BGK && p.collision != LBM_TRT) return "collision must be LBM_BGK or LBM_TRT";
    if (p.fluid_open != 0 && p.fluid_open != 1) return "fluid_open must be 0 or 1";
    if (p.ceq_field != 0 && p.ceq_field != 1) return "ceq_field must be 0 or 1";
    if (p.fluid_open) {
        if (p.inlet_axis < 0 || p.periodic[p.inlet_axis]) return "fluid_open needs inlet_axis >= 0 and that axis not periodic";
        if (!(p.rho_out > 0.0) || !(fabs(p.u_in) < 0.3)) return "fluid_open needs rho_out > 0 and |u_in| < 0.3";
    }
    return "";
}

int64_t default_links(const lbm_params &p) {
    const int64_t N = (int64_t)p.nx * p.ny * p.nz;
    int64_t m = p.max_links > 0 ? p.max_links : N * (p.fluid_q - 1) / 4;
    if (m < 4096) m = 4096;
    if (m > 2147483000LL) m = 2147483000LL;
    return m;
}

}  // namespace

namespace lbm {

// Carve the workspace for n domains.  With base == nullptr only the size is
// computed.
size_t workspace_layout(const lbm_params *p, int nd, Ctx *c, char *base) {
    long N = 0, R = 0, RW = 0;
    int64_t L = 0;
    for (int d = 0; d < nd; d++) {
        const long Nd = (long)p[d].nx * p[d].ny * p[d].nz;
        const long Rd = (long)p[d].ny * p[d].nz;
        N += Nd;
        R += Rd;
        RW += Rd * ((p[d].nx + 63) / 64);
        L += default_links(p[d]);
    }
    if (L > 2147483000LL) L = 2147483000LL;
    const int Q = p[0].fluid_q, QS = p[0].solute_q;
    const size_t ts = p[0].precision == LBM_FP64 ? 8 : 4;
    // direction stride: a multiple of 64 elements and an odd multiple of
    // 64 * ts bytes, so the 2Q streams of a step do not all start on the same
    // large power-of-two boundary
    long S = (N + 63) / 64 * 64;
    if ((S / 64) % 2 == 0) S += 64;
    // a task holds 64 nodes, or ends at a row (narrow rows: at most one task
    // per row ends early) or at a word-window limit (wide rows: advances at
    // least one word)
    const long task_cap = 2 * R + RW + N / 64 + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *r = base ? base + off : nullptr;
        off += up(bytes);
        return r;
    };
    char *f0 = take(ts * Q * S), *f1 = take(ts * Q * S), *g0 = take(ts * QS * S), *g1 = take(ts * QS * S);
    char *doms = take(sizeof(DomDev) * nd);
    char *noff = take(8 * (nd + 1)), *woff = take(8 * (nd + 1)), *roff = take(8 * (nd + 1));
    char *rows = take(sizeof(RowWord) * RW), *tasks = take(sizeof(Task) * task_cap);
    // per slot (S >= N entries): nodeof, lbase, and the scan temporaries
    char *nodeof = take(4 * S), *kof = take(4 * N), *lbase = take(4 * S);
    char *flags = take(4 * N), *rmask = take(4 * N), *cnt = take(4 * S), *sidx = take(4 * S);
    char *phi = take(8 * N), *kr = take(8 * N), *nrm = take(24 * N), *solid = take(N);
    char *phif = take(8 * S), *phis = take(8 * L);
    const bool ceqf = p[0].ceq_field != 0;
    char *ceq = take(ceqf ? 8 * N : 0), *lceq = take(ceqf ? ts * L : 0);
    char *lbeta = take(ts * L), *lq = take(ts * L), *lq2 = take(ts * L), *lnode = take(4 * L),
         *lsolid = take(4 * L), *ldir = take(L);
    char *sif = take(4 * L), *soff = take(4 * (L + 1)), *slinks = take(4 * L), *sdom = take(4 * L);
    char *bsum = take(4 * ((N + 4095) / 4096 + 64));
    char *dpart = take(16 * ((N + 255) / 256 + 1));
    char *dacc = take(8 * 64), *iacc = take(4 * 64), *fpart = take(8 * 2 * FOLD_G);
    const long nxp = (N + 255) / 256 + 1;
    char *xpart = take(8 * nxp), *xio = take(16 * task_cap);
    // phase change (single lattice): old compact map, candidates, records
    const bool pc = nd == 1 && p[0].phase_change != 0;
    const long ev_cap = pc ? (N < 65536 ? N : 65536) : 0;
    char *kof_old = take(pc ? 4 * N : 0), *evlist = take(4 * ev_cap);
    char *evrec = take(event_record_bytes() * ev_cap), *evmom = take(pc ? 16 * N : 0);
    char *evheap = take(4 * ev_cap);
    if (c && base) {
        c->kof_old = (int32_t *)kof_old;
        c->evlist = (int32_t *)evlist;
        c->evrec = evrec;
        c->evmom = evmom;
        c->evheap = (int32_t *)evheap;
        c->ev_cap = ev_cap;
        c->ev_capacity = false;
        c->N = N;
        c->S = S;
        c->R = R;
        c->RW = RW;
        c->Q = Q;
        c->ceq = ceqf ? (double *)ceq : nullptr;
        c->lceq = ceqf ? (void *)lceq : nullptr;
        c->ceq_set = false;
        c->QS = QS;
        c->red = QS != Q;
        c->smask = Q == 9 ? (c->red ? axis_mask<D2Q9>() : sol_mask<D2Q9, false>())
                          : (c->red ? axis_mask<D3Q19>() : sol_mask<D3Q19, false>());
        c->task_cap = task_cap;
        c->max_links = L;
        c->f[0] = f0; c->f[1] = f1; c->g[0] = g0; c->g[1] = g1;
        c->doms = (DomDev *)doms;
        c->dnode_off = (long *)noff; c->dword_off = (long *)woff; c->drow_off = (long *)roff;
        c->rows = (RowWord *)rows; c->tasks = (Task *)tasks;
        c->nodeof = (int32_t *)nodeof; c->kof = (int32_t *)kof; c->lbase = (int32_t *)lbase;
        c->flags = (uint32_t *)flags; c->rmask = (uint32_t *)rmask;
        c->cnt = (int32_t *)cnt; c->sidx = (int32_t *)sidx;
        c->phi = (double *)phi; c->kr = (double *)kr; c->nrm = (double *)nrm;
        c->phif = (double *)phif; c->phis = (double *)phis;
        c->phi_stale = false;
        c->solid = (uint8_t *)solid;
        c->lbeta = lbeta; c->lq = lq; c->lnode = (int32_t *)lnode; c->lsolid = (int32_t *)lsolid;
        c->lqb[0] = lq; c->lqb[1] = lq2; c->lq_next = 1;
        c->ldir = (uint8_t *)ldir;
        c->sif = (int32_t *)sif; c->soff = (int32_t *)soff; c->slinks = (int32_t *)slinks;
        c->sdom = (int32_t *)sdom;
        c->bsum = (int32_t *)bsum;
        c->dpart = (double *)dpart;
        c->dacc = (double *)dacc; c->iacc = (int32_t *)iacc; c->fpart = (double *)fpart;
        c->xpart = (double *)xpart; c->n_xpart = nxp;
        c->xio = (double *)xio;
    }
    return off;
}

}  // namespace lbm

// true when p is device memory the GPU can address (NULL counts as valid for
// optional arguments and is checked separately where required)
static bool dev_ptr_ok(const void *p) {
    if (!p) return true;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static lbm_status bad_ptr(Ctx *c, const char *what) {
    c->err = std::string(what) + " is not a device pointer";
    return LBM_EINVAL;
}

static lbm_status dev_err(Ctx *c, hipError_t e, const char *what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
}

// host view of domain d: box, rest-fraction weights and constants
static void setup_domain(const lbm_params &p, DomHost &d) {
    d.p = p;
    d.box.nx = p.nx;
    d.box.ny = p.ny;
    d.box.nz = p.nz;
    for (int a = 0; a < 3; a++) d.box.per[a] = p.periodic[a];
    d.box.shift = p.xwrap_shift_y;
    d.box.inlet_axis = p.inlet_axis;
    d.N = (long)p.nx * p.ny * p.nz;
    d.R = (long)p.ny * p.nz;
    d.W = (p.nx + 63) / 64;
    const double *w = p.fluid_q == 9 ? D2Q9::w : D3Q19::w;
    const double w0 = w[0];
    for (int i = 0; i < 19; i++) d.ws[i] = 0.0;
    if (p.solute_q != p.fluid_q) {
        // D2Q5 / D3Q7 (Sec. 2.2, eqs. RestFraction, RestFractionCs2): w_0 = J0,
        // every axis direction c_s^2 / 2, c_s^2 = (1 - J0)/dim; without a rest
        // fraction the common lattice, J0 = 1/3 (D2Q5) or 1/4 (D3Q7).  The
        // axis directions of the fluid lattice all weigh w_ax, so ws = w * wsc.
        const uint32_t m = p.fluid_q == 9 ? axis_mask<D2Q9>() : axis_mask<D3Q19>();
        const double j0 = p.j0 < 0 ? (p.dim == 2 ? 1.0 / 3.0 : 0.25) : p.j0;
        const double w_ax = p.fluid_q == 9 ? D2Q9::w[2] : D3Q19::w[1];
        d.cs2s = (1.0 - j0) / p.dim;
        d.wsc = 0.5 * d.cs2s / w_ax;
        d.ws[0] = j0;
        for (int i = 1; i < p.fluid_q; i++) d.ws[i] = (m >> i) & 1u ? w[i] * d.wsc : 0.0;
    } else if (p.j0 < 0) {
        for (int i = 0; i < p.fluid_q; i++) d.ws[i] = w[i];
        d.wsc = 1.0;
        d.cs2s = 1.0 / 3.0;
    } else {
        // rest fraction: w_0 = J0, moving weights and c_s^2 scaled by (1-J0)/(1-w0)
        const double sc = (1.0 - p.j0) / (1.0 - w0);
        d.ws[0] = p.j0;
        for (int i = 1; i < p.fluid_q; i++) d.ws[i] = w[i] * sc;
        d.wsc = sc;
        d.cs2s = sc / 3.0;
    }
    d.gamma = p.tau_ad / (p.tau_ad - 0.5);
}

static DomDev dom_record(const DomHost &h, bool fp64) {
    DomDev D;
    memset(&D, 0, sizeof D);
    const lbm_params &p = h.p;
    D.box = h.box;
    D.W = h.W;
    D.mech = p.rbc_mechanics;
    D.scheme = p.rbc_scheme;
    D.node_off = h.node_off;
    D.word_off = h.word_off;
    D.row_off = h.row_off;
    D.omega_f = 1.0 / p.tau_ns;
    D.omega_g = 1.0 / p.tau_ad;
    D.force_fac = 1.0 - 0.5 / p.tau_ns;
    // TRT: the second rate of each lattice from the magic parameter 3/16,
    // (tau+ - 1/2)(tau- - 1/2) = 3/16; BGK: both rates equal
    D.trt = p.collision == LBM_TRT;
    D.fopen = p.fluid_open;
    D.u_in = p.u_in;
    D.rho_out = p.rho_out;
    D.smask = p.solute_q == p.fluid_q ? (1u << p.fluid_q) - 1u
                                      : (p.fluid_q == 9 ? axis_mask<D2Q9>() : axis_mask<D3Q19>());
    const double tfm = 0.5 + (3.0 / 16.0) / (p.tau_ns - 0.5), tgm = 0.5 + (3.0 / 16.0) / (p.tau_ad - 0.5);
    D.omega_fm = D.trt ? 1.0 / tfm : D.omega_f;
    D.force_fac_m = 1.0 - 0.5 * D.omega_fm;
    D.omega_gs = D.trt ? 1.0 / tgm : D.omega_g;
    for (int a = 0; a < 3; a++) D.F[a] = p.force[a];
    for (int i = 0; i < 19; i++) D.ws[i] = h.ws[i];
    D.wsc = h.wsc;
    D.inv_cs2s = 1.0 / h.cs2s;
    D.cs2s = h.cs2s;
    D.gamma = h.gamma;
    D.rho0 = fp64 ? 0.0 : p.rho0;
    D.c_ref = fp64 ? 0.0 : p.c_ref;
    D.ceq_dev = p.c_eq - D.c_ref;
    D.c_in = p.inlet_axis >= 0 ? p.c_in : 0.0;
    D.vma = p.v_m * p.a_m;
    D.v_m = p.v_m;
    D.kr0 = p.k_r;
    return D;
}

static std::string check_batch(const lbm_params *p, int n) {
    if (n < 1) return "a batch needs at least one domain";
    for (int d = 0; d < n; d++) {
        std::string m = check_params(p[d]);
        if (!m.empty()) return (n > 1 ? "domain " + std::to_string(d) + ": " : std::string()) + m;
        if (p[d].dim != p[0].dim || p[d].fluid_q != p[0].fluid_q || p[d].solute_q != p[0].solute_q ||
            p[d].precision != p[0].precision || p[d].collision != p[0].collision ||
            p[d].fluid_open != p[0].fluid_open || p[d].ceq_field != p[0].ceq_field)
            return "all domains of a batch need the same dim, lattices, precision, collision, fluid_open "
                   "and ceq_field";
        if (p[d].phase_change != 0 && n > 1) return "phase_change is not supported in a batch";
        if (p[d].phase_change != 0 && p[d].phase_change != 1) return "phase_change must be 0 or 1";
    }
    double N = 0;
    for (int d = 0; d < n; d++) N += (double)p[d].nx * p[d].ny * p[d].nz;
    if (N >= 2147483647.0) return "the batch exceeds 2^31 - 1 nodes";
    return "";
}

static lbm_status create_common(const lbm_params *params, int nd, void *dev_workspace, size_t bytes,
                                void *hip_stream, lbm_ctx **out) {
    if (!params || !out) {
        g_create_err = "null argument";
        return LBM_EINVAL;
    }
    *out = nullptr;
    std::string m = check_batch(params, nd);
    if (!m.empty()) {
        g_create_err = m;
        return LBM_EINVAL;
    }
    const size_t need = workspace_layout(params, nd, nullptr, nullptr);
    if (!dev_workspace || bytes < need) {
        g_create_err = "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                       std::to_string(need) + " needed";
        return LBM_ENOMEM;
    }
    if (((uintptr_t)dev_workspace) % ALIGN != 0) {
        g_create_err = "workspace must be 256-byte aligned";
        return LBM_EINVAL;
    }
    if (!dev_ptr_ok(dev_workspace)) {
        g_create_err = "workspace is not device memory";
        return LBM_EINVAL;
    }
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) {
        g_create_err = "host allocation failed";
        return LBM_ENOMEM;
    }
    c->p = params[0];
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        g_create_err = "hipGetDevice failed";
        return LBM_EDEVICE;
    }
    c->dim = params[0].dim;
    c->fp64 = params[0].precision == LBM_FP64;
    c->ndom = nd;
    c->dom.resize(nd);
    long noff = 0, woff = 0, roff = 0;
    std::vector<long> hn(nd + 1), hw(nd + 1), hr(nd + 1);
    std::vector<DomDev> hd(nd);
    for (int d = 0; d < nd; d++) {
        DomHost &h = c->dom[d];
        setup_domain(params[d], h);
        h.node_off = noff;
        h.word_off = woff;
        h.row_off = roff;
        hn[d] = noff;
        hw[d] = woff;
        hr[d] = roff;
        noff += h.N;
        woff += h.R * h.W;
        roff += h.R;
        hd[d] = dom_record(h, c->fp64);
        if (params[d].inlet_axis >= 0) c->any_planes = true;
    }
    hn[nd] = noff;
    hw[nd] = woff;
    hr[nd] = roff;
    c->ws_bytes = bytes;
    workspace_layout(params, nd, c, (char *)dev_workspace);
    hipError_t e = hipMemcpy(c->doms, hd.data(), sizeof(DomDev) * nd, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->dnode_off, hn.data(), 8 * (nd + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->dword_off, hw.data(), 8 * (nd + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->drow_off, hr.data(), 8 * (nd + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        g_create_err = std::string("uploading the domain table: ") + hipGetErrorString(e);
        delete c;
        return LBM_EDEVICE;
    }
    c->cur = 0;
    c->n_links = c->n_sif = 0;
    c->step = c->n_events = 0;
    c->have_geom = c->have_state = false;
    c->have_events = false;
    c->cfg.wg_waves = 4;
    c->cfg.xcd_remap = 1;
    c->cfg.graph_steps = 0;
    c->cfg.overlap = 0;
    c->gexec = nullptr;
    c->graph_built = 0;
    c->geom_epoch = 0;
    c->have_side = false;
    c->phi_pending[0] = c->phi_pending[1] = false;
    c->last_phi = -1;
    {
        hipError_t es = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        bool ok = es == hipSuccess;
        int made = 0;
        for (int b = 0; ok && b < 2; b++) {
            ok = hipEventCreateWithFlags(&c->ev_stp[b], hipEventDisableTiming) == hipSuccess;
            if (ok) made++;
            ok = ok && hipEventCreateWithFlags(&c->ev_phi[b], hipEventDisableTiming) == hipSuccess;
            if (ok) made++;
            ok = ok && hipEventCreateWithFlags(&c->ev_adj[b], hipEventDisableTiming) == hipSuccess;
            if (ok) made++;
        }
        if (!ok) {   // run without the overlap
            (void)hipGetLastError();
            if (es == hipSuccess) (void)hipStreamDestroy(c->side);
            for (int b = 0; b < 2; b++) {
                if (made > 3 * b) (void)hipEventDestroy(c->ev_stp[b]);
                if (made > 3 * b + 1) (void)hipEventDestroy(c->ev_phi[b]);
                if (made > 3 * b + 2) (void)hipEventDestroy(c->ev_adj[b]);
            }
        }
        c->have_side = ok;
    }
    c->adj.valid = false;
    // the threshold flag of the phase-change steps starts clear (batch 0 is
    // never used)
    c->evbatch = c->evidx = 0;
    if (hipMemsetAsync(c->iacc + 16, 0, 8, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        lbm_destroy((lbm_ctx *)c);
        g_create_err = "could not clear the context's flags";
        return LBM_EDEVICE;
    }
    *out = (lbm_ctx *)c;
    return LBM_OK;
}

static void drop_graph(Ctx *c) {
    if (c->graph_built) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->graph_built = 0;
}

// Capture n (even) steps starting from buffer 0 on a private stream; the
// graph holds kernel launches only.
static hipError_t build_graph(Ctx *c, int n) {
    drop_graph(c);
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    const hipStream_t user = c->stream;
    const int cur = c->cur;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        c->stream = cs;
        c->cur = 0;
        const int lqn = c->lq_next;
        void *lq = c->lq;
        // inside the capture only waits on events recorded in it
        c->phi_pending[0] = c->phi_pending[1] = false;
        c->last_phi = -1;
        c->lq_next = 1;
        hipError_t le = hipSuccess;
        for (int t = 0; t < n && le == hipSuccess; t++) le = launch_step(*c, nullptr, c->have_side && c->cfg.overlap);
        if (le == hipSuccess) le = join_side(*c);
        c->stream = user;
        c->cur = cur;
        c->lq_next = lqn;
        c->lq = lq;
        c->phi_pending[0] = c->phi_pending[1] = false;
        c->last_phi = -1;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e == hipSuccess) c->graph_built = n;
    }
    (void)hipStreamDestroy(cs);
    return e;
}

// Phase change after a step: event pass, then (if anything changed) the
// geometry rebuilt in place and the populations moved to the new layout.
static hipError_t phase_change_pass(Ctx *c, bool flagged, bool *capacity) {
    int64_t nev = 0;
    bool ovf = false;
    hipError_t e = launch_events(*c, flagged, &nev, &ovf);
    if (e != hipSuccess) return e;
    if (ovf) *capacity = true;
    if (nev == 0) return hipSuccess;
    drop_graph(c);
    c->geom_epoch++;
    c->adj.valid = false;
    int64_t nl = 0, ns = 0;
    e = launch_geometry(*c, c->solid, c->nrm, c->kr, c->phi, &nl, &ns);
    if (e != hipSuccess) return e;
    if (nl > c->max_links) {
        *capacity = true;
        c->have_geom = c->have_state = false;
        return hipSuccess;
    }
    c->n_links = nl;
    c->n_sif = ns;
    e = launch_relayout(*c);
    c->n_events += nev;
    return e;
}

// Phase change: the launches of up to kmax steps are queued as one batch.
// Every kernel of the batch does nothing once an earlier step of the batch
// has crossed a threshold (the device flag), so the host waits once per
// batch; it then counts the steps done (the crossing one included), puts its
// buffer and exchange parities back to what they were after that step, and
// the event pass follows.  After values were set from outside a step (all
// working copies must be checked) the batch is one step.  On return *done
// steps have run and *flagged says whether the last one crossed.
static hipError_t phase_change_batch(Ctx *c, int kmax, int *done, bool *flagged, hipEvent_t *ev = nullptr) {
    const int K = c->full_check ? 1 : kmax;
    c->evbatch = c->evbatch >= 0x7ffffffe ? 1 : c->evbatch + 1;
    const int cur0 = c->cur, lq0 = c->lq_next;
    hipError_t e = hipSuccess;
    for (int j = 1; j <= K && e == hipSuccess; j++) {
        c->evidx = j;
        e = launch_step(*c, ev);
    }
    unsigned long long w = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&w, c->iacc + 16, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    *flagged = (int)(w >> 32) == c->evbatch;
    const int n = *flagged ? (int)(unsigned)w : K;
    c->cur = (n & 1) ? 1 - cur0 : cur0;
    c->lq_next = (n & 1) ? 1 - lq0 : lq0;
    c->lq = c->lqb[(n & 1) ? lq0 : 1 - lq0];
    c->step += n;
    *done = n;
    return hipSuccess;
}

// plain: kernel launches on the context stream only (no graph, which would
// allocate when built, and no second stream)
static hipError_t run_steps(Ctx *c, int32_t nsteps, bool plain = false) {
    int32_t t = 0;
    if (c->p.phase_change) {
        // events need a decision on the host (no graphs): batches of steps
        while (t < nsteps) {
            int done = 0;
            bool flagged = false, cap = false;
            const int kmax = nsteps - t < 32 ? (int)(nsteps - t) : 32;
            hipError_t e = phase_change_batch(c, kmax, &done, &flagged);
            if (e != hipSuccess) return e;
            t += done;
            e = phase_change_pass(c, flagged, &cap);
            if (e != hipSuccess) return e;
            if (cap) {
                c->err = "phase change exceeded a capacity (events per step or reactive links)";
                c->ev_capacity = true;
                return hipErrorOutOfMemory;
            }
        }
        return hipSuccess;
    }
    const int gs = plain ? 0 : (c->cfg.graph_steps + 1) & ~1;
    if (gs > 0 && nsteps >= gs) {
        if (c->cur != 0) {   // the graph starts from buffer 0
            hipError_t e = launch_step(*c);
            if (e != hipSuccess) return e;
            c->step++;
            t++;
        }
        if (nsteps - t >= gs) {
            if (c->graph_built != gs) {
                hipError_t e = build_graph(c, gs);
                if (e != hipSuccess) return e;
            }
            while (nsteps - t >= gs) {
                hipError_t e = join_side(*c);   // eager work before the graph
                if (e != hipSuccess) return e;
                e = hipGraphLaunch(c->gexec, c->stream);
                if (e != hipSuccess) return e;
                c->step += gs;
                t += gs;
                // the graph starts at buffer 1 and runs an even number of steps
                c->lq_next = 1;
                c->lq = c->lqb[0];
            }
        }
    }
    for (; t < nsteps; t++) {
        hipError_t e = launch_step(*c, nullptr, !plain && c->have_side && c->cfg.overlap);
        if (e != hipSuccess) return e;
        c->step++;
    }
    // every later operation on the context stream sees the solid fractions
    return join_side(*c);
}

static bool cfg_ok(const lbm_launch_config &g) {
    return (g.wg_waves == 1 || g.wg_waves == 2 || g.wg_waves == 4 || g.wg_waves == 8) &&
           (g.xcd_remap == 0 || g.xcd_remap == 1) && g.graph_steps >= 0 && g.graph_steps <= 100000 &&
           (g.overlap == 0 || g.overlap == 1);
}

extern "C" {

lbm_status lbm_workspace_bytes(const lbm_params *params, size_t *bytes) {
    return lbm_batch_workspace_bytes(params, 1, bytes);
}

lbm_status lbm_batch_workspace_bytes(const lbm_params *params, int32_t n, size_t *bytes) {
    if (!params || !bytes) return LBM_EINVAL;
    std::string m = check_batch(params, n);
    if (!m.empty()) {
        g_create_err = m;
        return LBM_EINVAL;
    }
    *bytes = workspace_layout(params, n, nullptr, nullptr);
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params *params, void *dev_workspace, size_t bytes, void *hip_stream,
                      lbm_ctx **out) {
    return create_common(params, 1, dev_workspace, bytes, hip_stream, out);
}

lbm_status lbm_create_batch(const lbm_params *params, int32_t n, void *dev_workspace, size_t bytes,
                            void *hip_stream, lbm_ctx **out) {
    return create_common(params, n, dev_workspace, bytes, hip_stream, out);
}

lbm_status lbm_batch_offsets(const lbm_ctx *ctx, int64_t *node_off) {
    const Ctx *c = (const Ctx *)ctx;
    if (!c || !node_off) return LBM_EINVAL;
    for (int d = 0; d < c->ndom; d++) node_off[d] = c->dom[d].node_off;
    node_off[c->ndom] = c->N;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *ctx) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return;
    if (c->have_events)
        for (int k = 0; k < 4; k++) (void)hipEventDestroy(c->ev[k]);
    drop_graph(c);
    if (c->have_side) {
        (void)hipStreamSynchronize(c->side);
        for (int b = 0; b < 2; b++) {
            (void)hipEventDestroy(c->ev_stp[b]);
            (void)hipEventDestroy(c->ev_phi[b]);
            (void)hipEventDestroy(c->ev_adj[b]);
        }
        (void)hipStreamDestroy(c->side);
    }
    delete c;
}

const char *lbm_last_error(const lbm_ctx *ctx) {
    if (!ctx) return g_create_err.c_str();
    return ((const Ctx *)ctx)->err.c_str();
}

lbm_status lbm_set_ceq(lbm_ctx *ctx, const double *c_eq) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (!c->ceq) {
        c->err = "lbm_set_ceq needs a context created with ceq_field = 1";
        return LBM_EINVAL;
    }
    if (!c_eq) {
        c->err = "c_eq is required";
        return LBM_EINVAL;
    }
    if (!dev_ptr_ok(c_eq)) return bad_ptr(c, "c_eq");
    hipError_t e = hipMemcpyAsync(c->ceq, c_eq, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return dev_err(c, e, "lbm_set_ceq");
    c->ceq_set = true;
    return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_ctx *ctx, const uint8_t *solid, const double *normals,
                            const double *k_r, const double *phi0) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (!solid) {
        c->err = "solid mask is required";
        return LBM_EINVAL;
    }
    if (!dev_ptr_ok(solid)) return bad_ptr(c, "solid");
    if (!dev_ptr_ok(normals)) return bad_ptr(c, "normals");
    if (!dev_ptr_ok(k_r)) return bad_ptr(c, "k_r");
    if (!dev_ptr_ok(phi0)) return bad_ptr(c, "phi0");
    int64_t nl = 0, ns = 0;
    drop_graph(c);
    c->geom_epoch++;
    hipError_t e = launch_geometry(*c, solid, normals, k_r, phi0, &nl, &ns);
    if (e != hipSuccess) return dev_err(c, e, "geometry preparation");
    if (nl > c->max_links) {
        c->err = "geometry has " + std::to_string(nl) + " reactive links; params.max_links allows " +
                 std::to_string(c->max_links);
        c->have_geom = false;
        return LBM_ECAPACITY;
    }
    c->n_links = nl;
    c->n_sif = ns;
    c->have_geom = true;
    c->have_state = false;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx *ctx, const double *rho, const double *u, const double *cc) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (!c->have_geom) {
        c->err = "lbm_init_fields before lbm_set_geometry";
        return LBM_ESTATE;
    }
    if (!dev_ptr_ok(rho)) return bad_ptr(c, "rho");
    if (!dev_ptr_ok(u)) return bad_ptr(c, "u");
    if (!dev_ptr_ok(cc)) return bad_ptr(c, "c");
    hipError_t e = launch_init(*c, rho, u, cc);
    if (e != hipSuccess) return dev_err(c, e, "init");
    c->step = 0;
    c->adj.valid = false;
    c->have_state = true;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) {
        c->err = "nsteps must be >= 0";
        return LBM_EINVAL;
    }
    if (!c->have_state) {
        c->err = "lbm_step before lbm_init_fields";
        return LBM_ESTATE;
    }
    hipError_t e = run_steps(c, nsteps);
    if (c->ev_capacity) {
        c->ev_capacity = false;
        return LBM_ECAPACITY;
    }
    if (e != hipSuccess) return dev_err(c, e, "step launch");
    return LBM_OK;
}

lbm_status lbm_set_launch_config(lbm_ctx *ctx, const lbm_launch_config *cfg) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !cfg) return LBM_EINVAL;
    if (!cfg_ok(*cfg)) {
        c->err = "launch config: wg_waves in {1,2,4,8}, xcd_remap in {0,1}, "
                 "0 <= graph_steps <= 100000, overlap in {0,1}";
        return LBM_EINVAL;
    }
    if (cfg->wg_waves != c->cfg.wg_waves || cfg->xcd_remap != c->cfg.xcd_remap ||
        cfg->overlap != c->cfg.overlap)
        drop_graph(c);
    c->cfg = *cfg;
    return LBM_OK;
}

lbm_status lbm_get_launch_config(const lbm_ctx *ctx, lbm_launch_config *cfg) {
    const Ctx *c = (const Ctx *)ctx;
    if (!c || !cfg) return LBM_EINVAL;
    *cfg = c->cfg;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *ctx, int32_t trial_steps, lbm_launch_config *best,
                        double *ms_per_step, int64_t *steps_run) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (trial_steps < 1 || trial_steps > 100000) {
        c->err = "trial_steps must be in 1..100000";
        return LBM_EINVAL;
    }
    if (!c->have_state) {
        c->err = "lbm_autotune before lbm_init_fields";
        return LBM_ESTATE;
    }
    const int64_t step0 = c->step;
    const lbm_launch_config keep = c->cfg;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return dev_err(c, e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return dev_err(c, e, "hipEventCreate");
    }
    // time n steps under configuration g after w untimed steps
    auto trial = [&](const lbm_launch_config &g, int w, int n, double *ms) -> hipError_t {
        if (g.wg_waves != c->cfg.wg_waves || g.xcd_remap != c->cfg.xcd_remap ||
            g.overlap != c->cfg.overlap)
            drop_graph(c);
        c->cfg = g;
        hipError_t r = run_steps(c, w);
        if (r == hipSuccess) r = hipEventRecord(e0, c->stream);
        if (r == hipSuccess) r = run_steps(c, n);
        if (r == hipSuccess) r = hipEventRecord(e1, c->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float t = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&t, e0, e1);
        *ms = (double)t / n;
        return r;
    };
    lbm_launch_config bc = keep;
    double bms = 1e300;
    const int waves[4] = {1, 2, 4, 8};
    // an open channel or a per-node C_eq always runs the 4-wave tile
    const bool fixed_tile = c->p.fluid_open != 0 || c->lceq != nullptr;
    for (int wi = 0; wi < 4 && e == hipSuccess; wi++)
        for (int rm = 0; rm < 2 && e == hipSuccess; rm++) {
            if (fixed_tile && waves[wi] != 4) continue;
            lbm_launch_config g = {waves[wi], rm, 0, 0};
            double ms = 0.0;
            e = trial(g, 2, trial_steps, &ms);
            if (e == hipSuccess && ms < bms) {
                bms = ms;
                bc = g;
            }
        }
    if (e == hipSuccess && c->have_side && !c->p.phase_change) {
        lbm_launch_config g = bc;
        g.overlap = 1;
        double ms = 0.0;
        e = trial(g, 2, trial_steps, &ms);
        if (e == hipSuccess && ms < bms) {
            bms = ms;
            bc = g;
        }
    }
    const int gsteps[3] = {16, 64, 256};
    for (int gi = 0; gi < 3 && e == hipSuccess; gi++) {
        const int gs = gsteps[gi];
        if (gs > 4 * trial_steps) break;
        lbm_launch_config g = bc;
        g.graph_steps = gs;
        const int n = ((trial_steps + gs - 1) / gs) * gs;
        double ms = 0.0;
        e = trial(g, gs + 1, n, &ms);   // the untimed part builds the graph
        if (e == hipSuccess && ms < bms) {
            bms = ms;
            bc = g;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        drop_graph(c);
        c->cfg = keep;
        return dev_err(c, e, "autotune");
    }
    if (bc.wg_waves != c->cfg.wg_waves || bc.xcd_remap != c->cfg.xcd_remap ||
        bc.overlap != c->cfg.overlap)
        drop_graph(c);
    c->cfg = bc;
    if (best) *best = bc;
    if (ms_per_step) *ms_per_step = bms;
    if (steps_run) *steps_run = c->step - step0;
    return LBM_OK;
}

lbm_status lbm_step_timed(lbm_ctx *ctx, int32_t nsteps, double *ms) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !ms || nsteps < 0) return LBM_EINVAL;
    if (!c->have_state) {
        c->err = "lbm_step_timed before lbm_init_fields";
        return LBM_ESTATE;
    }
    if (!c->have_events) {
        for (int k = 0; k < 4; k++) {
            hipError_t e = hipEventCreate(&c->ev[k]);
            if (e != hipSuccess) return dev_err(c, e, "hipEventCreate");
        }
        c->have_events = true;
    }
    ms[0] = ms[1] = 0.0;
    for (int32_t t = 0; t < nsteps; t++) {
        hipError_t e = hipSuccess;
        bool flagged = false;
        if (c->p.phase_change) {
            int done = 0;
            e = phase_change_batch(c, 1, &done, &flagged, c->ev);
        } else {
            e = launch_step(*c, c->ev);
            c->step++;
        }
        if (e != hipSuccess) return dev_err(c, e, "step launch");
        e = hipEventSynchronize(c->ev[3]);
        if (e != hipSuccess) return dev_err(c, e, "event sync");
        float a = 0.f, b = 0.f;
        e = hipEventElapsedTime(&a, c->ev[0], c->ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, c->ev[2], c->ev[3]);
        if (e != hipSuccess) return dev_err(c, e, "event timing");
        ms[0] += a;
        ms[1] += b;
        if (c->p.phase_change) {
            bool cap = false;
            e = phase_change_pass(c, flagged, &cap);
            if (e != hipSuccess) return dev_err(c, e, "phase change");
            if (cap) {
                c->err = "phase change exceeded a capacity (events per step or reactive links)";
                return LBM_ECAPACITY;
            }
        }
    }
    return LBM_OK;
}

static size_t adj_layout(const Ctx *c, int64_t nsteps, int64_t ckpt, AdjState *st, char *base) {
    const size_t ts = c->fp64 ? 8 : 4;
    const size_t slot = (size_t)c->QS * (size_t)c->S * ts;
    const size_t ncp = (size_t)((nsteps + ckpt - 1) / ckpt);
    size_t off = 0;
    auto take = [&](size_t n) -> char * {
        char *p = base ? base + off : nullptr;
        off += (n + ALIGN - 1) / ALIGN * ALIGN;
        return p;
    };
    // per step of a segment, one source value per reactive link of the
    // current geometry (which a recorded run keeps)
    const size_t stride = ((size_t)c->n_links + 1 + 63) / 64 * 64;
    char *ck = take(ncp * slot);
    char *r0 = take(slot), *r1 = take(slot);
    char *ls = take((size_t)ckpt * stride * ts);
    char *ls2 = ncp > 1 ? take((size_t)ckpt * stride * ts) : nullptr;
    char *p0 = take(slot), *p1 = take(slot);
    char *gb = take(sizeof(double) * (size_t)(c->max_links + 1));
    if (st) {
        st->ckpt = ck;
        st->rst[0] = r0;
        st->rst[1] = r1;
        st->lsrc = ls;
        st->lsrc2 = ls2;
        st->src_stride = (int64_t)stride;
        st->p[0] = p0;
        st->p[1] = p1;
        st->gbeta = (double *)gb;
    }
    return off;
}

static lbm_status adj_check(Ctx *c, int32_t nsteps, int32_t ckpt) {
    if (nsteps < 1 || ckpt < 1 || ckpt > nsteps) {
        c->err = "need 1 <= ckpt_every <= nsteps";
        return LBM_EINVAL;
    }
    if (c->ndom != 1) {
        c->err = "the adjoint works on single-lattice contexts";
        return LBM_EINVAL;
    }
    if (c->p.inlet_axis >= 0 || c->p.phase_change) {
        c->err = "the adjoint needs inlet_axis = -1 and phase_change = 0";
        return LBM_EINVAL;
    }
    if (c->p.force[0] != 0.0 || c->p.force[1] != 0.0 || c->p.force[2] != 0.0) {
        c->err = "the adjoint needs the fluid at rest (no body force)";
        return LBM_EINVAL;
    }
    if (c->ceq) {
        c->err = "the adjoint takes a uniform c_eq (ceq_field = 0)";
        return LBM_EINVAL;
    }
    return LBM_OK;
}

lbm_status lbm_adjoint_workspace_bytes(const lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every,
                                       size_t *bytes) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !bytes) return LBM_EINVAL;
    lbm_status st = adj_check(c, nsteps, ckpt_every);
    if (st != LBM_OK) return st;
    *bytes = adj_layout(c, nsteps, ckpt_every, nullptr, nullptr);
    return LBM_OK;
}

// checks shared by lbm_record and lbm_record_static, up to the workspace
static lbm_status record_check(Ctx *c, int32_t nsteps, int32_t ckpt_every) {
    lbm_status st = adj_check(c, nsteps, ckpt_every);
    if (st != LBM_OK) return st;
    if (!c->have_state) {
        c->err = "lbm_record before lbm_init_fields";
        return LBM_ESTATE;
    }
    return LBM_OK;
}

// the recorded run into the adjoint workspace at base (checked by the caller)
static lbm_status record_into(Ctx *c, int32_t nsteps, int32_t ckpt_every, char *base, bool plain) {
    bool rest = false;
    hipError_t e = launch_rest_check(*c, &rest);
    if (e != hipSuccess) return dev_err(c, e, "rest check");
    if (!rest) {
        c->err = "the adjoint needs the fluid at rest: every fluid node at the equilibrium at "
                 "rest of one common density";
        return LBM_EINVAL;
    }
    c->adj.valid = false;
    adj_layout(c, nsteps, ckpt_every, &c->adj, base);
    const size_t slot = (size_t)c->QS * (size_t)c->S * (c->fp64 ? 8 : 4);
    for (int32_t t = 0; t < nsteps; t += ckpt_every) {
        e = hipMemcpyAsync((char *)c->adj.ckpt + (size_t)(t / ckpt_every) * slot, c->g[c->cur], slot,
                           hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return dev_err(c, e, "checkpoint copy");
        e = run_steps(c, nsteps - t < ckpt_every ? nsteps - t : ckpt_every, plain);
        if (e != hipSuccess) return dev_err(c, e, "step launch");
    }
    c->adj.nsteps = nsteps;
    c->adj.ckpt_every = ckpt_every;
    c->adj.end_step = c->step;
    c->adj.geom_epoch = c->geom_epoch;
    c->adj.static_gen = 0;
    c->adj.valid = true;
    return LBM_OK;
}

lbm_status lbm_record(lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every, void *dev_workspace,
                      size_t bytes) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    lbm_status st = record_check(c, nsteps, ckpt_every);
    if (st != LBM_OK) return st;
    const size_t need = adj_layout(c, nsteps, ckpt_every, nullptr, nullptr);
    if (!dev_workspace || bytes < need) {
        c->err = "adjoint workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                 std::to_string(need) + " needed";
        return LBM_ENOMEM;
    }
    if (((uintptr_t)dev_workspace) % ALIGN != 0 || !dev_ptr_ok(dev_workspace)) {
        c->err = "adjoint workspace must be 256-byte aligned device memory";
        return LBM_EINVAL;
    }
    return record_into(c, nsteps, ckpt_every, (char *)dev_workspace, false);
}

// ---------------------------------------------------------------------------
// lbm_record_static: the adjoint workspace in a device array of the library.
// In host code `scratch` only stands for the array; its device address on
// each GPU comes from hipGetSymbolAddress, taken once per device (that
// device current) and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[LBM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];
int64_t scratch_gen[MAX_DEVICES];   // records taken into each device's array
}  // namespace

lbm_status lbm_record_static(lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    lbm_status st = record_check(c, nsteps, ckpt_every);
    if (st != LBM_OK) return st;
    const size_t need = adj_layout(c, nsteps, ckpt_every, nullptr, nullptr);
    if (need > (size_t)LBM_STATIC_SCRATCH_BYTES) {
        c->err = "the recorded run needs " + std::to_string(need) + " bytes, more than the " +
                 std::to_string((size_t)LBM_STATIC_SCRATCH_BYTES) +
                 " of the library's static array (use lbm_record with a workspace)";
        return LBM_ENOMEM;
    }
    const int dev = c->device;
    if (dev < 0 || dev >= MAX_DEVICES) {
        c->err = "device index out of range for the static array";
        return LBM_EINVAL;
    }
    char *base = nullptr;
    int64_t gen = 0;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (!scratch_ptr[dev]) {
            int prev = -1;
            hipError_t e = hipGetDevice(&prev);
            if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
            void *ptr = nullptr;
            if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
            if (e != hipSuccess || !ptr) return dev_err(c, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                        "hipGetSymbolAddress of the static array");
            scratch_ptr[dev] = ptr;
        }
        base = (char *)scratch_ptr[dev];
        gen = ++scratch_gen[dev];
    }
    st = record_into(c, nsteps, ckpt_every, base, true);
    if (st == LBM_OK) c->adj.static_gen = gen;
    return st;
}

static lbm_status adjoint_common(Ctx *c, const double *dL_dC, double *grad_k, double *ms);

lbm_status lbm_adjoint(lbm_ctx *ctx, const double *dL_dC, double *grad_k) {
    return adjoint_common((Ctx *)ctx, dL_dC, grad_k, nullptr);
}

lbm_status lbm_adjoint_timed(lbm_ctx *ctx, const double *dL_dC, double *grad_k, double *ms) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !ms) return LBM_EINVAL;
    if (!c->have_events) {
        for (int k = 0; k < 4; k++) {
            hipError_t e = hipEventCreate(&c->ev[k]);
            if (e != hipSuccess) return dev_err(c, e, "hipEventCreate");
        }
        c->have_events = true;
    }
    ms[0] = ms[1] = ms[2] = 0.0;
    return adjoint_common(c, dL_dC, grad_k, ms);
}

static lbm_status adjoint_common(Ctx *c, const double *dL_dC, double *grad_k, double *ms) {
    if (!c) return LBM_EINVAL;
    if (!dL_dC || !grad_k) {
        c->err = "dL_dC and grad_k are required";
        return LBM_EINVAL;
    }
    if (!dev_ptr_ok(dL_dC)) return bad_ptr(c, "dL_dC");
    if (!dev_ptr_ok(grad_k)) return bad_ptr(c, "grad_k");
    if (!c->adj.valid || c->adj.end_step != c->step || c->adj.geom_epoch != c->geom_epoch) {
        c->err = "no recorded run ends at the current state (call lbm_record first)";
        return LBM_ESTATE;
    }
    if (c->adj.static_gen != 0) {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (scratch_gen[c->device] != c->adj.static_gen) {
            c->err = "a later lbm_record_static on this GPU has overwritten the recorded run";
            return LBM_ESTATE;
        }
    }
    hipError_t e = launch_adjoint(*c, dL_dC, grad_k, ms);
    if (e != hipSuccess) return dev_err(c, e, "adjoint");
    return LBM_OK;
}

lbm_status lbm_get_fields(lbm_ctx *ctx, double *rho, double *u, double *cc, double *phi,
                          uint8_t *type) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (!c->have_state) {
        c->err = "no state: call lbm_init_fields first";
        return LBM_ESTATE;
    }
    if (!dev_ptr_ok(rho)) return bad_ptr(c, "rho");
    if (!dev_ptr_ok(u)) return bad_ptr(c, "u");
    if (!dev_ptr_ok(cc)) return bad_ptr(c, "c");
    if (!dev_ptr_ok(phi)) return bad_ptr(c, "phi");
    if (!dev_ptr_ok(type)) return bad_ptr(c, "type");
    hipError_t e = launch_fields(*c, rho, u, cc, phi, type);
    if (e != hipSuccess) return dev_err(c, e, "get_fields");
    return LBM_OK;
}

lbm_status lbm_get_pops(lbm_ctx *ctx, double *f, double *g) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return LBM_EINVAL;
    if (!c->have_state) {
        c->err = "no state: call lbm_init_fields first";
        return LBM_ESTATE;
    }
    if (!dev_ptr_ok(f)) return bad_ptr(c, "f");
    if (!dev_ptr_ok(g)) return bad_ptr(c, "g");
    hipError_t e = launch_pops(*c, f, g);
    if (e != hipSuccess) return dev_err(c, e, "get_pops");
    return LBM_OK;
}

lbm_status lbm_get_exchange(lbm_ctx *ctx, double *q) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !q) return LBM_EINVAL;
    if (!c->have_geom) {
        c->err = "no geometry";
        return LBM_ESTATE;
    }
    if (!dev_ptr_ok(q)) return bad_ptr(c, "q");
    hipError_t e = launch_exchange(*c, q);
    if (e != hipSuccess) return dev_err(c, e, "get_exchange");
    return LBM_OK;
}

lbm_status lbm_get_diag(lbm_ctx *ctx, lbm_diag *out) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !out) return LBM_EINVAL;
    if (!c->have_state) {
        c->err = "no state: call lbm_init_fields first";
        return LBM_ESTATE;
    }
    double sums[5] = {0, 0, 0, 0, 0};
    int32_t nan_flag = 0;
    hipError_t e = launch_diag(*c, sums, &nan_flag);
    if (e != hipSuccess) return dev_err(c, e, "diag");
    memset(out, 0, sizeof *out);
    out->step = c->step;
    out->n_events = c->n_events;
    out->n_links = c->n_links;
    out->n_solid_iface = c->n_sif;
    out->n_fluid = c->n_fluid;
    out->n_fluid_iface = c->n_fluid_iface;
    out->wall_exchange = sums[0];
    out->mass_c = sums[1];
    out->phi_sum = sums[2];
    out->inlet_exchange = sums[3];
    out->outlet_exchange = sums[4];
    out->n_tasks = c->n_tasks;
    out->n_row_words = c->RW;
    out->nan_flag = nan_flag;
    if (nan_flag) {
        c->err = "non-finite population";
        return LBM_ENUMERIC;
    }
    return LBM_OK;
}

// state layout: header | f (Q*S of T) | g (QS*S of T), both in the blocked
// population layout | phi | kr (N doubles) | nrm (3N doubles) | solid (N bytes)
struct StateHeader {
    uint64_t magic;
    int64_t N, Q, precision, step, n_events;
    double wall_ex;
    int64_t QS;
    double inlet_ex, outlet_ex;
};

lbm_status lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes) {
    const Ctx *c = (const Ctx *)ctx;
    if (!c || !bytes) return LBM_EINVAL;
    const size_t ts = c->fp64 ? 8 : 4;
    *bytes = sizeof(StateHeader) + ts * (c->Q + c->QS) * c->S + 8 * 5 * c->N + c->N;
    return LBM_OK;
}

lbm_status lbm_save_state(lbm_ctx *ctx, void *dev_buf, size_t bytes) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !dev_buf) return LBM_EINVAL;
    size_t need = 0;
    lbm_state_bytes(ctx, &need);
    if (bytes < need) {
        c->err = "state buffer too small";
        return LBM_ENOMEM;
    }
    if (!c->have_state) {
        c->err = "no state to save";
        return LBM_ESTATE;
    }
    if (!dev_ptr_ok(dev_buf)) return bad_ptr(c, "state buffer");
    const size_t ts = c->fp64 ? 8 : 4;
    StateHeader h;
    memset(&h, 0, sizeof h);
    h.magic = 0x4c424d5242433033ULL;
    h.N = c->N; h.Q = c->Q; h.QS = c->QS; h.precision = c->p.precision; h.step = c->step;
    h.n_events = c->n_events;
    double acc[5] = {0, 0, 0, 0, 0};
    hipError_t e = launch_fold_exchange(*c);
    if (e == hipSuccess) e = launch_phi_flush(*c);
    if (e == hipSuccess) e = hipMemcpyAsync(acc, c->dacc, sizeof acc, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_err(c, e, "save_state");
    h.wall_ex = acc[0];
    h.inlet_ex = acc[3];
    h.outlet_ex = acc[4];
    char *b = (char *)dev_buf;
    e = hipMemcpyAsync(b, &h, sizeof h, hipMemcpyHostToDevice, c->stream);
    size_t off = sizeof h;
    const size_t fb = ts * c->Q * c->S, gb = ts * c->QS * c->S;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->f[c->cur], fb, hipMemcpyDeviceToDevice, c->stream);
    off += fb;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->g[c->cur], gb, hipMemcpyDeviceToDevice, c->stream);
    off += gb;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->phi, 8 * c->N, hipMemcpyDeviceToDevice, c->stream);
    off += 8 * c->N;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->kr, 8 * c->N, hipMemcpyDeviceToDevice, c->stream);
    off += 8 * c->N;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->nrm, 24 * c->N, hipMemcpyDeviceToDevice, c->stream);
    off += 24 * c->N;
    if (e == hipSuccess) e = hipMemcpyAsync(b + off, c->solid, c->N, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_err(c, e, "save_state");
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx *ctx, const void *dev_buf, size_t bytes) {
    Ctx *c = (Ctx *)ctx;
    if (!c || !dev_buf) return LBM_EINVAL;
    size_t need = 0;
    lbm_state_bytes(ctx, &need);
    if (bytes < need) {
        c->err = "state buffer too small";
        return LBM_ENOMEM;
    }
    if (!dev_ptr_ok(dev_buf)) return bad_ptr(c, "state buffer");
    StateHeader h;
    const char *b = (const char *)dev_buf;
    hipError_t e = hipMemcpyAsync(&h, b, sizeof h, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_err(c, e, "load_state");
    if (h.magic != 0x4c424d5242433033ULL || h.N != c->N || h.Q != c->Q || h.QS != c->QS ||
        h.precision != c->p.precision) {
        c->err = "state buffer does not match this context";
        return LBM_EINVAL;
    }
    const size_t ts = c->fp64 ? 8 : 4;
    const size_t fb = ts * c->Q * c->S, gb = ts * c->QS * c->S;
    const size_t pops = sizeof h, phio = pops + fb + gb;
    // geometry first (rebuilds links from solid, normals and k_r), then state
    const double *phi_src = (const double *)(b + phio);
    const double *kr_src = (const double *)(b + phio + 8 * c->N);
    const double *nrm_src = (const double *)(b + phio + 16 * c->N);
    const uint8_t *sol_src = (const uint8_t *)(b + phio + 40 * c->N);
    int64_t nl = 0, ns = 0;
    drop_graph(c);
    c->geom_epoch++;
    c->adj.valid = false;
    e = launch_geometry(*c, sol_src, nrm_src, kr_src, phi_src, &nl, &ns);
    if (e != hipSuccess) return dev_err(c, e, "load_state geometry");
    if (nl > c->max_links) {
        c->err = "saved geometry exceeds max_links";
        return LBM_ECAPACITY;
    }
    c->n_links = nl;
    c->n_sif = ns;
    c->have_geom = true;
    c->cur = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(c->f[0], b + pops, fb, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->g[0], b + pops + fb, gb, hipMemcpyDeviceToDevice, c->stream);
    // the cumulative exchanges (the diag sums in between are recomputed)
    double acc[5] = {h.wall_ex, 0.0, 0.0, h.inlet_ex, h.outlet_ex};
    if (e == hipSuccess) e = hipMemcpyAsync(c->dacc, acc, sizeof acc, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_zero_exchange(*c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_err(c, e, "load_state");
    c->step = h.step;
    c->n_events = h.n_events;
    c->have_state = true;
    return LBM_OK;
}

}  // extern "C"
