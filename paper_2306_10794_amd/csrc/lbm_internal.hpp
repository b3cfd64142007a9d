// lbm_internal.hpp -- context layout and kernel launchers shared by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbmrbc.h"
#include "lbm_device.hpp"

namespace lbm {

// Per-step kernel arguments (passed by value; lives in the kernarg segment).
template <typename T>
struct StepArgs {
    const T *__restrict__ fin;
    T *__restrict__ fout;
    const T *__restrict__ gin;
    T *__restrict__ gout;
    const Task *__restrict__ tasks;
    const RowWord *__restrict__ rows;
    const DomDev *__restrict__ doms;
    const int32_t *__restrict__ nodeof;  // compact index -> dense node
    const int32_t *__restrict__ lbase;   // compact index -> links of the nodes before it
    const T *__restrict__ lbeta;         // per link: (1 - k)/(1 + k)
    T *__restrict__ lq;                  // per link: mass exchanged in this step
    double *__restrict__ phif;           // [S] solid fraction of fluid nodes, compact order
    const T *__restrict__ lceq;          // per link: C_eq - C_ref of its solid node (per-node C_eq)
    double *__restrict__ xio;            // [2][task_cap] per task: inlet, outlet exchange (cumulative)
    // phase change (else evflag is null): the step's kernels set *evflag to
    // (evbatch << 32 | evidx) when an interface node's solid fraction is past
    // a threshold, and do nothing at all once a step of the same batch before
    // this one (index < evidx) has set it
    unsigned long long *evflag;
    int32_t evbatch, evidx;
    long task_cap;
    long ntasks;
    long S;                              // stride between directions
    int ndom;                            // domains of the context
};

// host view of one domain
struct DomHost {
    lbm_params p;
    Box box;
    long N, R, node_off, word_off, row_off;
    int W;
    double gamma, cs2s, ws[19], wsc;
    int64_t links_cap;
};

// recorded forward run for the adjoint (memory in a caller workspace)
struct AdjState {
    bool valid;
    int64_t nsteps, ckpt_every, end_step, geom_epoch;
    int64_t static_gen;      // > 0: the run lives in the library's static array,
                             // as the static_gen-th record taken into it
    void *ckpt;              // [ceil(nsteps/ckpt_every)][Q][S] solute states
    void *rst[2];            // [Q][S] recomputed states (alternating)
    void *lsrc;              // [ckpt_every][n_links + 1] per step and reactive link: the
                             // source value of its rate condition (recomputed)
    void *lsrc2;             // a second such buffer (runs of more than one segment,
                             // else null): the next segment is recomputed into it
                             // while the transposed steps read the first
    int64_t src_stride;      // elements between two steps of lsrc
    void *p[2];              // [Q][S] adjoint arrays
    double *gbeta;           // [max_links] dL/dbeta
};

// workgroups of the first level of the fixed-order folds (exchange totals,
// diagnostics)
constexpr int FOLD_G = 64;

struct Ctx {
    lbm_params p;            // parameters of domain 0 (precision, lattice)
    lbm_launch_config cfg;   // tile / schedule of the step launches
    hipStream_t stream;
    int device;              // HIP device current at lbm_create
    int Q, dim;
    int QS;                  // solute directions (Q, or 5 / 7 on D2Q5 / D3Q7)
    bool red;                // the solute runs on the reduced set (QS < Q)
    uint32_t smask;          // solute set as a mask over the fluid directions
    int ndom;
    std::vector<DomHost> dom;
    long N;                  // nodes of all domains
    long S;                  // stride between directions of the compact arrays
    long R;                  // rows of all domains
    long RW;                 // row words of all domains
    long task_cap;
    bool fp64;
    int64_t max_links;
    // device arrays carved from the caller workspace
    void *f[2], *g[2];       // populations, f [Q][S], g [QS][S] (T = double or float), compact
    DomDev *doms;            // [ndom]
    long *dnode_off;         // [ndom + 1] dense node offsets
    long *dword_off;         // [ndom + 1] row-word offsets
    long *drow_off;          // [ndom + 1] row offsets
    RowWord *rows;           // [RW]
    Task *tasks;             // [task_cap]
    int32_t *nodeof;         // [N] compact -> dense
    int32_t *kof;            // [N] dense -> compact (-1 for solid)
    int32_t *lbase;          // [N] compact -> first link
    uint32_t *flags, *rmask; // [N] dense geometry flags / reactive-link bits
    int32_t *cnt;            // scratch [N]
    int32_t *sidx;           // scratch [N]
    double *phi, *kr, *nrm;  // [N], [N], [N][3]
    // working copies of the solid fraction that the step kernels update with
    // coalesced accesses: fluid nodes in compact order, solid interface nodes
    // in solid-side order; phi[] is brought up to date from them (flush)
    // before anything reads it, and they are refilled from phi[] (gather)
    // whenever the geometry is rebuilt
    double *phif, *phis;     // [S], [max_links]
    bool phi_stale;          // phi[] lags the working copies
    uint8_t *solid;          // [N]
    double *ceq;             // [N] per-node C_eq (ceq_field contexts), else null
    void *lceq;              // [max_links] of T: C_eq - C_ref per link, else null
    bool ceq_set;            // lbm_set_ceq has filled ceq
    void *lbeta, *lq;        // [max_links] of T; lq: exchanges of the last step
    void *lqb[2];            // the two exchange buffers lq alternates between
    int lq_next;             // buffer the next step writes
    // overlap of the solid-side phi kernel of step t with the fused kernel of
    // step t + 1 (second stream; default priority)
    hipStream_t side;
    hipEvent_t ev_stp[2], ev_phi[2];
    hipEvent_t ev_adj[2];    // the adjoint's recomputation on the side stream
    bool have_side;
    bool phi_pending[2];     // ev_phi[b] marks a solid-side kernel still to be waited for
    int last_phi;            // buffer of the last overlapped solid-side kernel, -1 none
    int32_t *lnode, *lsolid; // [max_links]
    uint8_t *ldir;           // [max_links]
    int32_t *sif, *soff, *slinks; // solid interface list [max_links], offsets [max_links+1], [max_links]
    int32_t *sdom;           // [max_links] domain of each solid interface node
    double *fpart;           // [2 * FOLD_G] first-level sums of the fixed-order folds
    int32_t *bsum;           // scan scratch
    int32_t *kof_old;        // [N] phase change: compact map before the events
    int32_t *evlist;         // [ev_cap] phase-change candidates in node order
    void *evrec;             // [ev_cap] event records
    void *evmom;             // [N] moments (C, rho) of every node before an event pass
    int32_t *evheap;         // [ev_cap] pending nodes of a pass, once they outgrow the LDS
    long ev_cap;
    bool full_check;         // the next threshold check scans every working copy
    int32_t evbatch, evidx;  // current batch of steps and step within it (threshold flag)
    bool ev_capacity;        // the last step ran out of event or link capacity
    double *dpart;           // per-workgroup partial sums of the reductions
    double *dacc;            // device accumulators: [0] wall exchange, [1..2] diag sums
    bool any_planes;         // some domain has an inlet and an outlet plane
    double *xio;             // [2][task_cap] inlet / outlet exchange of the tasks on those
                             // planes, one slot per task, folded into dacc[3..4] when read
    double *xpart;           // [n_xpart] wall exchange of the solid-side workgroups, one
                             // slot per workgroup, folded into dacc[0] when read
    long n_xpart;
    int32_t *iacc;           // device int accumulators
    size_t ws_bytes;
    int cur;                 // buffer holding the current state
    int64_t n_links, n_sif, n_fluid, n_fluid_iface, n_tasks;
    int64_t n_slots;         // population slots in use: 64 per task (each task's
                             // nodes in a 64-aligned block of its own), or
                             // n_fluid when that would not fit S
    int64_t step, n_events;
    bool have_geom, have_state;
    hipEvent_t ev[4];
    bool have_events;
    // graph of cfg.graph_steps steps (even), valid while the geometry and the
    // launch configuration are unchanged; replayed from buffer 0
    hipGraphExec_t gexec;
    int graph_built;         // steps in gexec, 0 = none
    int64_t geom_epoch;      // counts geometry changes
    AdjState adj;
    std::string err;
};

size_t workspace_layout(const lbm_params *p, int n, Ctx *c, char *base);

// launchers (return hipError_t of the first failing launch)
// ev: optional 4 events recorded around the two kernels of the step
hipError_t launch_step(Ctx &c, hipEvent_t *ev = nullptr, bool overlap = false);
// make the context stream wait for an overlapped solid-side kernel
hipError_t join_side(Ctx &c);
hipError_t launch_geometry(Ctx &c, const uint8_t *solid, const double *normals, const double *k_r,
                           const double *phi0, int64_t *n_links, int64_t *n_sif);
hipError_t launch_init(Ctx &c, const double *rho, const double *u, const double *cc);
hipError_t launch_fields(Ctx &c, double *rho, double *u, double *cc, double *phi, uint8_t *type);
hipError_t launch_pops(Ctx &c, double *f, double *g);
hipError_t launch_exchange(Ctx &c, double *q);
hipError_t launch_diag(Ctx &c, double *sums, int32_t *nan_flag);
hipError_t launch_fold_exchange(Ctx &c);
hipError_t launch_phi_gather(Ctx &c, long nf, long nsif);
hipError_t launch_phi_flush(Ctx &c);
hipError_t launch_zero_exchange(Ctx &c);
hipError_t launch_rest_check(Ctx &c, bool *at_rest);
hipError_t launch_events(Ctx &c, bool flagged, int64_t *n_events, bool *overflow);
hipError_t launch_relayout(Ctx &c);
size_t event_record_bytes();
// ms (optional, host array of 2): summed durations of the recomputation and of
// the transposed-step kernels (each launch timed with events; synchronises)
hipError_t launch_adjoint(Ctx &c, const double *dldc, double *grad, double *ms = nullptr);
hipError_t scan_excl(Ctx &c, const int32_t *in, int32_t *out, long n, int32_t *total_dev);

}  // namespace lbm
