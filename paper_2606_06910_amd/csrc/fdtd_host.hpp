// fdtd_host.hpp -- host-side context of the C ABI (shared by the API,
// adjoint and autotuner translation units).
#pragma once
#include "../../include/fdtd.h"
#include "fdtd_dev.hpp"

#include <map>
#include <string>
#include <utility>
#include <vector>

constexpr int kOFF = 128;   // leading pad of every field (elements)
constexpr int kTYMAX = 64;  // tallest y tile (rows) a kernel may overhang
constexpr int kMaxRec = 65536;  // receivers per shot with temporal blocking
constexpr int kTimingClasses = 6;   // update, psi, record, exchange, band update, temporal block
constexpr int kBandTX = BAND_TX, kBandZ = 32;   // band-kernel tile width and z chunk
constexpr int kCUs = 256;   // compute units of an MI355X (the default z-march plan shares them)
constexpr long kSmallShot = 150L * 150 * 150;   // a lone shot below this many points runs naive by default

struct ShotH {
    fdtd_shot_config c;
    int nx = 0, ny = 0, nz = 0;
    int gy = 0, gz = 0;        // ghost (loopback) axes
    int s = 1, g = 4;          // exchange interval and ghost depth
    int fy = 4, fz = 4;        // frame rows / planes
    int P = 0, PY = 0, S = 0;  // row pitch, rows per plane, plane stride (elements)
    size_t elems = 0;          // elements per field buffer
    size_t esz = 4;            // bytes per stored field element
    int Llo[3] = {0, 0, 0}, Lhi[3] = {0, 0, 0};
    int LX = 0, LY = 0, LZ = 0, nmax = 0;
    int WX = 0;                 // x psi/zeta row width: max(Llo[0], Lhi[0])
    int SY = 0, SZ = 0;         // y, z psi/zeta strides: slab width + 1 zero slot (0 without layers)
    size_t psi_elems[3] = {0, 0, 0};
    // workspace offsets
    size_t o_u[4] = {0, 0, 0, 0}, o_d = 0, o_m = 0, o_psi[3] = {0, 0, 0}, o_zeta[3] = {0, 0, 0}, o_prof = 0;
    size_t o_work = 0, o_xbuf = 0, xbuf_bytes = 0;
    size_t o_jobs[2][4] = {};
    int njobs[2][4] = {};
    long jobmax[2][4] = {};
    int nwork = 0;
    size_t o_band = 0;         // band-kernel tile list, all box kinds (for the largest compute box)
    int nband = 0;
    // model / source / receivers
    bool vel_set = false;
    double vmax = 0, vref = 0, scale = 1;
    bool has_src = false;
    const float *wav = nullptr;
    int src_nt = 0, sx = 0, sy = 0, sz = 0;
    float amp = 0;
    const int32_t *rec = nullptr;
    int nrec = 0;
    float *traces = nullptr;
    int cap = 0;
    // plan
    int variant = FDTD_VARIANT_ZMARCH, ry = 2, zchunk = 64, tk = 1;
    int zcols = 1;             // z-march x points per lane (1: 64-wide tiles, 2: 128-wide tiles)
    // temporal blocking (FP32, Dirichlet, single-shot contexts): 4 level buffers,
    // interior box B (outside every band, x bounds multiples of 4), tile list over B_K,
    // receivers sorted by z
    bool tb_bufs = false;
    int blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    size_t o_tbwork = 0, o_reczs = 0, o_recix = 0;
    int ntbwork = 0, tb_zchunk = 64;
    // checkpoints / adjoint
    int ck_every = 0, ck_count = 0, ck_nt = 0;
    char *ck_buf = nullptr;
    size_t ck_bytes = 0;
};

struct fdtd_ctx {
    std::vector<ShotH> shots;
    std::vector<DevShot> hdesc;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
    hipStream_t side = nullptr;         // second stream: interior update concurrent with psi + band
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // adjoint: reverse sweep of one segment on its own stream while the main
    // stream recomputes the next segment's levels (double-buffered)
    hipStream_t adj_stream = nullptr;
    hipEvent_t ev_adj[5] = {};          // ready[2], free[2], join
    bool single_stream = false;         // never create the side stream (everything on `stream`)
    char *ws = nullptr;
    size_t ws_bytes = 0, need = 0;
    size_t o_stepc = 0, o_scratch = 0, o_desc = 0, o_work_all = 0, o_band_all = 0;
    int nwork_all = 0, nband_all = 0;
    // multi-shot z-march launches: one per distinct (ry, zchunk) plan
    struct Group {
        int ry, zchunk, cols;
        size_t off;   // offset into the o_work_all region (items)
        int nwork;
    };
    std::vector<Group> groups;
    int storage = 0;
    int band_ty = BAND_TY;    // band-kernel tile rows: BAND_TY_TALL for one shot of 2^27 points or more
    int sentinel_every = 0;   // > 0: scan the newest level for NaN/Inf after every such step (scratch slot 3)
    int iu = 0;         // level buffer holding u^n
    int ium1 = 1;       // level buffer holding u^{n-1} (FP32) -- 16-bit keeps d^n in its own buffer
    long step = 0;
    bool saving = true; // checkpoint saving enabled (off during adjoint recomputation)
    std::string err;
    unsigned char state_hdr[1024] = {};  // header of the last fdtd_save_state (read by its copy)
    struct GraphEntry {
        hipGraphExec_t exec;
        int end_iu, end_ium1;
    };
    std::map<std::pair<long, long>, GraphEntry> graphs;
    // per-kernel-class event timing (eager stepping only)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[kTimingClasses];
    double t_sum[kTimingClasses] = {};
    long t_cnt[kTimingClasses] = {};
};

// Element offset of (x, y, z) = (0, 0, 0) from the start of a field buffer of
// the shot (every field, m and the adjoint's full-grid arrays share it); row
// starts, and so x = 0, are 64-element aligned.
inline size_t origin_elems(const ShotH &s) {
    return (size_t)kOFF + (size_t)s.fz * s.S + (size_t)s.fy * s.P;
}

// helpers exported by fdtd_api.hip for the other translation units
size_t fdtd_state_bytes(const ShotH &s);
char *fdtd_ws(fdtd_ctx *ctx, size_t off);
void fdtd_enqueue_step_shot(fdtd_ctx *ctx, int shot);
void fdtd_restore_state(fdtd_ctx *ctx, int i, char *ck);
void *fdtd_field_origin(fdtd_ctx *ctx, const ShotH &s, size_t off);
float *fdtd_m_origin(fdtd_ctx *ctx, const ShotH &s);
int fdtd_rewrite_work(fdtd_ctx *ctx);
int fdtd_reupload(fdtd_ctx *ctx);
int fdtd_ready(fdtd_ctx *ctx);
int fdtd_zero_state(fdtd_ctx *ctx);
void fdtd_set_copy_vec(CopyJob &j);

inline void fdtd_clear_graphs(fdtd_ctx *ctx) {
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.second.exec);
    ctx->graphs.clear();
}
