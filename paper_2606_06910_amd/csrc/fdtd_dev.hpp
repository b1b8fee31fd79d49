// fdtd_dev.hpp -- device-side definitions shared by the gfx950 kernels.
//
// Per-point arithmetic of the second-order acoustic leapfrog with the
// kappa-inclusive CPML of the paper's section "CPML Boundary Layers"
// (stretched derivative (1/kappa) D f + psi applied twice):
//   psi_d  <- b psi_d + a D1_d u                        (slab points, pre-pass)
//   eta_d   = kinv D2_d u + dkinv D1_d u + D1_d psi_d   (slab + 4-cell band)
//   zeta_d <- b zeta_d + a eta_d                        (slab points)
//   Lt_d    = kinv eta_d + zeta_d
//   u^{n+1} = (2 u^n - u^{n-1}) + m * sum_d Lt_d   (+ m * source)
// Every kernel variant evaluates a point through the functions below, in the
// same operation order, so variants agree bit for bit.  Compiled with
// -ffp-contract=off: every fused multiply-add is written out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FDTD_R 4          // stencil radius
#define FDTD_MAXSHOTS 64

// ---------------------------------------------------------------------------
// storage types: FP32, FP16 (_Float16) and BF16 (__bf16); arithmetic is FP32.
// ---------------------------------------------------------------------------
template <typename T> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
    static __device__ __forceinline__ float4 ld4(const float *p) { return *(const float4 *)p; }
    static __device__ __forceinline__ void st4(float *p, float4 v) { *(float4 *)p = v; }
};
template <> struct Store<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16 *p) { return (float)*p; }
    static __device__ __forceinline__ void st(_Float16 *p, float v) { *p = (_Float16)v; }
    static __device__ __forceinline__ float4 ld4(const _Float16 *p) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        h4 v = *(const h4 *)p;
        return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
    }
    static __device__ __forceinline__ void st4(_Float16 *p, float4 v) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        h4 o;
        o.x = (_Float16)v.x;
        o.y = (_Float16)v.y;
        o.z = (_Float16)v.z;
        o.w = (_Float16)v.w;
        *(h4 *)p = o;
    }
};
template <> struct Store<__bf16> {
    static __device__ __forceinline__ float ld(const __bf16 *p) { return (float)*p; }
    static __device__ __forceinline__ void st(__bf16 *p, float v) { *p = (__bf16)v; }
    static __device__ __forceinline__ float4 ld4(const __bf16 *p) {
        typedef __bf16 b4 __attribute__((ext_vector_type(4)));
        b4 v = *(const b4 *)p;
        return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
    }
    static __device__ __forceinline__ void st4(__bf16 *p, float4 v) {
        typedef __bf16 b4 __attribute__((ext_vector_type(4)));
        b4 o;
        o.x = (__bf16)v.x;
        o.y = (__bf16)v.y;
        o.z = (__bf16)v.z;
        o.w = (__bf16)v.w;
        *(b4 *)p = o;
    }
};

// ---------------------------------------------------------------------------
// One shot as the kernels see it (device-resident; read with uniform loads).
// Field element (x, y, z), -4 <= x < nx+4, -fy <= y < ny+fy, -fz <= z < nz+fz,
// is at  origin + z*S + y*P + x  in both level buffers and in m.
// ---------------------------------------------------------------------------
struct DevShot {
    void *u[4];            // level buffers (origin-adjusted), storage type T; [2], [3] only with temporal blocking
    void *dinc;            // 16-bit storage only: d^n = u^n - u^{n-1} (origin-adjusted); null for FP32
    const float *m;        // v^2 dt^2 (origin-adjusted), 0 in the frame
    float *psi[3];         // layer memory, compact slab layouts (see psi_index)
    float *zeta[3];
    const float *prof;     // [3][4][nmax]: b, a, kinv, dkinv per axis index
    const float *wav;      // source wavelet (borrowed), may be null
    float *traces;         // [cap][nrec] or null
    const int32_t *rec;    // [nrec][3] or null
    float src_scale;       // amplitude * storage_scale / (hx hy hz)
    float inv_scale;       // 1 / storage_scale
    int src_nt, sx, sy, sz;
    int nrec, trace_cap;
    int nx, ny, nz, P, PY, S, fy, fz;
    int Llo[3], Lhi[3];
    int LX, LY, LZ, nmax;
    int WX;                // x layer arrays: row width, max(Llo[0], Lhi[0])
    int SY, SZ;            // y, z layer arrays: strides along the slab axis, width + 1 slot that stays zero
    int ghost[3];          // 1 if the axis has ghost (loopback) faces
    int fused;             // 1: the band kernel advances psi_x and psi_z itself, the psi pass only psi_y
    float cc;              // sum_d (c0 + 2 c1) / h_d^2
    float w2[3][5];        // (c0 + 2 c1) / h_d^2, then c_l / h_d^2 for l = 1..4
    float w1[3][5];        // d_l / h_d   (w1[d][0] unused)
};

// Strided box copy (ghost pack/unpack).  Rows (ex elements) are copied in
// vb-byte pieces: vb in {16, 8, 4, 2} divides both row starts, every stride
// and the row length in bytes (set by the host, copy_vec_bytes).
struct CopyJob {
    const void *src;
    void *dst;
    int esz;              // bytes per element (2 or 4)
    int ex, ey, ez;       // box extent (elements)
    long sy, sz, dy, dz;  // row / plane strides (elements) of source and destination
    int vb;               // bytes per copied piece
};

// Roles of the level buffers in one launch and an optional box of points the
// launch leaves alone (inner region advanced by the temporal-blocking kernel).
struct Roles {
    int iu;          // buffer holding u^n
    int ium1;        // buffer holding u^{n-1} (FP32 storage)
    int iout;        // buffer receiving u^{n+1} (== ium1 for the in-place step)
    int ext;         // ghost-box extension of this sub-step
    int lo[3], hi[3];  // exclusion box [lo, hi) per axis; empty when lo >= hi on any axis
};
__device__ __forceinline__ bool in_box(const Roles &R, int x, int y, int z) {
    return x >= R.lo[0] && x < R.hi[0] && y >= R.lo[1] && y < R.hi[1] && z >= R.lo[2] && z < R.hi[2];
}

// Work item of the z-marching kernels: shot, x tile, y tile, z chunk.
struct WorkItem {
    int shot, tx, ty, zc;
};

// Work item of the band kernel: shot, band box, x tile, y tile, z chunk.
#define BAND_TX 32
#define BAND_TY 8          // tile rows (BAND_TX x BAND_TY threads), and
#define BAND_TY_TALL 16    // those of the taller tiles of large single-shot contexts
struct BandItem {
    int shot, box, tx, ty, zc, pad0, pad1, pad2;
};

// The band region of a shot (layer slabs plus the 4-cell margin their psi
// derivative reaches) within its compute box (extended by `ext` on ghost
// axes) as six disjoint boxes [lo, hi), k = 0..5:
//   0, 1  z below / above the non-band z range, all x and y
//   2, 3  y below / above the non-band y range, inside the non-band z range
//   4, 5  x below / above the non-band x range, inside the non-band y, z ranges
// and k = 6, the non-band box itself.  Along each axis the non-band range is
// [a, b): a = min(lo + 4, n) with a low layer (else the box start), b =
// max(n - hi - 4, a) with a high layer (else the box end), so that c < a or
// c >= b is exactly the band test (band_range returns a, b and the box
// extent [e0, e1) of one axis).
__host__ __device__ inline void band_range(int n, int Llo, int Lhi, int ghost, int ext, int &a, int &b, int &e0,
                                           int &e1) {
    e0 = ghost ? -ext : 0;
    e1 = n + (ghost ? ext : 0);
    a = Llo > 0 ? (Llo + FDTD_R < n ? Llo + FDTD_R : n) : e0;
    b = Lhi > 0 ? (n - Lhi - FDTD_R > a ? n - Lhi - FDTD_R : a) : e1;
}
// Along x the non-band range is narrowed to whole band tiles where a band fits
// one: [a, b) becomes [BAND_TX, b') with b' = max(b rounded down to a multiple
// of BAND_TX, n - BAND_TX), so that each x band box is one tile wide with every
// lane busy, and the non-band range starts on a 128-byte line (and, when n is
// a multiple of BAND_TX, ends on one).  The points between the band and the
// new bounds lie in no band; the band kernel gives them the interior
// arithmetic.  Where the two boxes would overlap, the range stays [a, b).
__host__ __device__ inline void band_range_x(int n, int Llo, int Lhi, int &a, int &b, int &e0, int &e1) {
    band_range(n, Llo, Lhi, 0, 0, a, b, e0, e1);
    int a2 = a, b2 = b;
    if (Llo > 0 && a <= BAND_TX) a2 = BAND_TX;
    if (Lhi > 0 && n - b <= BAND_TX) {
        const int r = b / BAND_TX * BAND_TX;
        b2 = r > n - BAND_TX ? r : n - BAND_TX;
    }
    if (a2 <= b2) {
        a = a2;
        b = b2;
    }
}
__host__ __device__ inline void band_box(const int n[3], const int Llo[3], const int Lhi[3], const int ghost[3],
                                         int ext, int k, int lo[3], int hi[3]) {
    int a[3], b[3];
    band_range_x(n[0], Llo[0], Lhi[0], a[0], b[0], lo[0], hi[0]);
    for (int d = 1; d < 3; ++d) band_range(n[d], Llo[d], Lhi[d], ghost[d], ext, a[d], b[d], lo[d], hi[d]);
    if (k == 6) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = a[d];
            hi[d] = b[d];
        }
    } else if (k == 0) {
        hi[2] = a[2];
    } else if (k == 1) {
        lo[2] = b[2];
    } else {
        lo[2] = a[2];
        hi[2] = b[2];
        if (k == 2) {
            hi[1] = a[1];
        } else if (k == 3) {
            lo[1] = b[1];
        } else {
            lo[1] = a[1];
            hi[1] = b[1];
            if (k == 4) hi[0] = a[0];
            else lo[0] = b[0];
        }
    }
}

// x tiles of band box k (box extent [lo0, hi0) along x): BAND_TX wide from the
// box start, except that boxes spanning all x (k < 4) cut their tiling at the
// start of the high x band, so that the band up to the end of x is a tile
// row of its own.  Returns the number of tiles; tile tx covers [x0, x1).
__host__ __device__ inline int band_xtiles(int nx, int Llo, int Lhi, int k, int lo0, int hi0, int tx, int *x0,
                                           int *x1) {
    int cut = hi0;
    if (k < 4) {
        int a, b, e0, e1;
        band_range_x(nx, Llo, Lhi, a, b, e0, e1);
        if (b > lo0 && b < hi0) cut = b;
    }
    const int nlo = (cut - lo0 + BAND_TX - 1) / BAND_TX;
    const int nhi = (hi0 - cut + BAND_TX - 1) / BAND_TX;
    if (tx < nlo) {
        *x0 = lo0 + tx * BAND_TX;
        *x1 = *x0 + BAND_TX < cut ? *x0 + BAND_TX : cut;
    } else {
        *x0 = cut + (tx - nlo) * BAND_TX;
        *x1 = *x0 + BAND_TX < hi0 ? *x0 + BAND_TX : hi0;
    }
    return nlo + nhi;
}

// LDS plane of a band-kernel tile of ty rows: its BAND_TX x ty points and a
// 4-cell halo on each side along x and y (corners unused), slot (column c,
// row r) = r * kBandLW + c, plus a dummy slot for lanes without a halo value.
constexpr int kBandLW = BAND_TX + 2 * FDTD_R;
__host__ __device__ constexpr int band_lds(int ty) { return kBandLW * (ty + 2 * FDTD_R) + 1; }
// The halo value lane t of a tile of ty rows stages: k = 0 one of the 4 rows
// above or below the tile (lanes below 2 * 4 * BAND_TX), k = 1 one of the 4
// columns left or right of it (lanes below 2 * 4 * ty).  (c, r): its slot;
// c = -1 when the lane has none.
__host__ __device__ inline void band_halo(int t, int k, int ty, int &c, int &r) {
    if (k == 0) {
        if (t >= 2 * FDTD_R * BAND_TX) {
            c = r = -1;
            return;
        }
        const int q = t / BAND_TX;
        r = q < FDTD_R ? q : q + ty;
        c = FDTD_R + t % BAND_TX;
        return;
    }
    if (t >= 2 * FDTD_R * ty) {
        c = r = -1;
        return;
    }
    const int j = t % (2 * FDTD_R);
    r = FDTD_R + t / (2 * FDTD_R);
    c = j < FDTD_R ? j : BAND_TX + j;
}

// ---------------------------------------------------------------------------
// layer geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_slab(int c, int n, int lo, int hi) {
    return (c < lo) || (c >= n - hi);
}
__device__ __forceinline__ bool in_band(int c, int n, int lo, int hi) {
    return (lo > 0 && c < lo + FDTD_R) || (hi > 0 && c >= n - hi - FDTD_R);
}
// slab index along an axis of width lo+hi (valid only when in_slab)
__device__ __forceinline__ int slab_pos(int c, int n, int lo, int hi) {
    return c < lo ? c : lo + (c - (n - hi));
}
// element index of (x, y, z) in the compact psi/zeta array of axis d:
//   x [side][z+fz][y+fy][WX]: side 0 the low layer (position x), side 1 the
//     high layer (position x - (nx - Lhi)), so that a tile row of one layer
//     is contiguous;
//   y [z+fz][SY][nx] and z [SZ][y+fy][nx], slab position LY (LZ) being an
//     extra slot that is never written and reads zero.
__device__ __forceinline__ long psi_index(const DevShot &s, int d, int x, int y, int z) {
    if (d == 0) {
        const long row = ((long)(z + s.fz) * s.PY + (y + s.fy)) * s.WX;
        if (x < s.Llo[0]) return row + x;
        return (long)(s.nz + 2 * s.fz) * s.PY * s.WX + row + (x - (s.nx - s.Lhi[0]));
    }
    if (d == 1) return ((long)(z + s.fz) * s.SY + slab_pos(y, s.ny, s.Llo[1], s.Lhi[1])) * s.nx + x;
    return ((long)slab_pos(z, s.nz, s.Llo[2], s.Lhi[2]) * s.PY + (y + s.fy)) * s.nx + x;
}
__device__ __forceinline__ int coord_n(const DevShot &s, int d) { return d == 0 ? s.nx : (d == 1 ? s.ny : s.nz); }

// psi_d at (x,y,z), zero outside the slab of axis d (and outside [0,n) along d)
__device__ __forceinline__ float psi_at(const DevShot &s, int d, int x, int y, int z) {
    int c = d == 0 ? x : (d == 1 ? y : z);
    int n = coord_n(s, d);
    if (c < 0 || c >= n || !in_slab(c, n, s.Llo[d], s.Lhi[d])) return 0.0f;
    return s.psi[d][psi_index(s, d, x, y, z)];
}

__device__ __forceinline__ float prof_at(const DevShot &s, int d, int f, int c) {
    return s.prof[(d * 4 + f) * s.nmax + c];
}

// ---------------------------------------------------------------------------
// stencil arithmetic (operation order is part of the contract)
// lo[l-1] = f(c - l), hi[l-1] = f(c + l), l = 1..4
//
// The nearest pair enters as differences from the centre,
//   D2 f = (c0 + 2 c1) f_c + c1 ((f_{+1} - f_c) + (f_{-1} - f_c)) + sum_{l>=2} c_l (f_{+l} + f_{-l}),
// (all weights / h^2), which is the same operator but keeps FP32 round-off
// from the large c0 f_c / 2 c1 f_c cancellation out of smooth fields; the
// weight array w2 holds (c0 + 2 c1)/h^2 in slot 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float pairs2(const float *w, float c, const float lo[4], const float hi[4], float acc) {
    acc = fmaf(w[1], (hi[0] - c) + (lo[0] - c), acc);
    acc = fmaf(w[2], lo[1] + hi[1], acc);
    acc = fmaf(w[3], lo[2] + hi[2], acc);
    acc = fmaf(w[4], lo[3] + hi[3], acc);
    return acc;
}
__device__ __forceinline__ float d2_axis(const float *w, float c, const float lo[4], const float hi[4]) {
    return pairs2(w, c, lo, hi, w[0] * c);
}
__device__ __forceinline__ float d1_axis(const float *w, const float lo[4], const float hi[4]) {
    float acc = w[1] * (hi[0] - lo[0]);
    acc = fmaf(w[2], hi[1] - lo[1], acc);
    acc = fmaf(w[3], hi[2] - lo[2], acc);
    acc = fmaf(w[4], hi[3] - lo[3], acc);
    return acc;
}
// interior points (outside every band): cc*c + x pairs + y pairs + z pairs,
// cc = sum_d w2[d][0]
// stencil weights of a shot held in registers (loaded once per kernel)
struct Coef {
    float cc;
    float w2[3][5];
};
__device__ __forceinline__ Coef load_coef(const DevShot &s) {
    Coef k;
    k.cc = s.cc;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < 5; ++l) k.w2[d][l] = s.w2[d][l];
    return k;
}
__device__ __forceinline__ float lap_interior(const Coef &k, float c, const float xl[4], const float xh[4],
                                              const float yl[4], const float yh[4], const float zl[4],
                                              const float zh[4]) {
    float acc = k.cc * c;
    acc = pairs2(k.w2[0], c, xl, xh, acc);
    acc = pairs2(k.w2[1], c, yl, yh, acc);
    acc = pairs2(k.w2[2], c, zl, zh, acc);
    return acc;
}
__device__ __forceinline__ float lap_interior(const DevShot &s, float c, const float xl[4], const float xh[4],
                                              const float yl[4], const float yh[4], const float zl[4],
                                              const float zh[4]) {
    float acc = s.cc * c;
    acc = pairs2(s.w2[0], c, xl, xh, acc);
    acc = pairs2(s.w2[1], c, yl, yh, acc);
    acc = pairs2(s.w2[2], c, zl, zh, acc);
    return acc;
}

// Buffer-resource access: a uniform base (scalar descriptor), a 32-bit byte
// offset per lane and a uniform 32-bit byte offset.  Offsets stay below 2^31.
typedef __amdgpu_buffer_rsrc_t Rsrc;
// A lane offset at or past a descriptor's record count reads zero and drops a
// store without touching memory; lanes that need no data use this one (any
// scalar offset the kernels add keeps the sum below 2^32).  Only the lane
// offset is range-checked: the scalar offset is not, so it must always
// address memory inside the buffer and never carries this value.
constexpr uint32_t kBufSkip = 0x80000000u;
__device__ __forceinline__ Rsrc make_rsrc(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, 0x7fffffff, 0x00020000);
}
// Field stores carry the non-temporal hint (cache-policy bit `nt`): a level
// written in one step is read only in the next, long after it has left the
// caches, so it need not displace the lines the other streams are re-reading.
// (Measured on the overlapped step: 768^3 FP32 2.17 -> 2.09 ms, 512^3 about
// 1 % faster.)  Loads of a stream read once per step (the second state and m
// of the z-march) take it too (ldnt): 512^3 0.693 -> 0.666 ms, 768^3 FP32
// 2.09 -> 1.97 ms.  u^n, whose lines the neighbouring tiles re-read through
// L2, keeps plain loads: the hint on every load made the 512^3 step 16 %
// slower.
constexpr int kStoreNT = 2, kLoadNT = 2;
template <typename T> struct Buf;
template <> struct Buf<float> {
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ float ldnt(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, kLoadNT));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, kStoreNT);
    }
};
template <> struct Buf<_Float16> {
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t vo, uint32_t so) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    static __device__ __forceinline__ float ldnt(Rsrc r, uint32_t vo, uint32_t so) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, kLoadNT));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, vo, so, kStoreNT);
    }
};
template <> struct Buf<__bf16> {
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t vo, uint32_t so) {
        return (float)__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    static __device__ __forceinline__ float ldnt(Rsrc r, uint32_t vo, uint32_t so) {
        return (float)__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, kLoadNT));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (__bf16)v), r, vo, so, kStoreNT);
    }
};

// Two consecutive x elements (an even element offset, so that the pair is 8-
// (FP32) or 4-byte (16-bit) aligned) loaded with one buffer load and widened
// to FP32.  The scalar offset must stay in range as for Buf.  (The 64-bit
// load is reinterpreted whole: taking its two elements one by one makes the
// compiler emit a single-dword load and repeat it in both.)
template <typename T> struct Buf2;
template <> struct Buf2<float> {
    static __device__ __forceinline__ float2 ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
};
template <> struct Buf2<_Float16> {
    static __device__ __forceinline__ float2 ld(Rsrc r, uint32_t vo, uint32_t so) {
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
        return make_float2((float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu)),
                           (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16)));
    }
};
template <> struct Buf2<__bf16> {
    static __device__ __forceinline__ float2 ld(Rsrc r, uint32_t vo, uint32_t so) {
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
        return make_float2((float)__builtin_bit_cast(__bf16, (unsigned short)(v & 0xffffu)),
                           (float)__builtin_bit_cast(__bf16, (unsigned short)(v >> 16)));
    }
};

// layer term of one axis given the old zeta (slab points); returns Lt_d and
// the new zeta in *zeta_new (slab points only)
__device__ __forceinline__ float cpml_axis(float d2, float d1, float dpsi, float kinv, float dkinv, float a,
                                           float b, bool slab, float zeta_old, float *zeta_new) {
    float eta = fmaf(kinv, d2, fmaf(dkinv, d1, dpsi));
    float z = 0.0f;
    if (slab) {
        z = fmaf(b, zeta_old, a * eta);
        *zeta_new = z;
    }
    return fmaf(kinv, eta, z);
}
__device__ __forceinline__ float leapfrog(float m, float lt, float c, float um1) {
    return fmaf(m, lt, fmaf(2.0f, c, -um1));
}
__device__ __forceinline__ float psi_update(float b, float psi, float a, float d1) {
    return fmaf(b, psi, a * d1);
}

// Layer-aware Laplacian of one point whose neighbours are given; reads psi
// neighbours, profiles and zeta from memory (all of them before any
// arithmetic, so that the loads are in flight together) and writes zeta back.
// Returns sum_d Lt_d (lap_interior when the point is outside every band).
__device__ __forceinline__ float lap_point(const DevShot &s, int x, int y, int z, float c, const float xl[4],
                                           const float xh[4], const float yl[4], const float yh[4],
                                           const float zl[4], const float zh[4]) {
    const bool bx = in_band(x, s.nx, s.Llo[0], s.Lhi[0]);
    const bool by = in_band(y, s.ny, s.Llo[1], s.Lhi[1]);
    const bool bz = in_band(z, s.nz, s.Llo[2], s.Lhi[2]);
    if (!(bx || by || bz)) return lap_interior(s, c, xl, xh, yl, yh, zl, zh);
    const float *lo[3] = {xl, yl, zl};
    const float *hi[3] = {xh, yh, zh};
    const bool band[3] = {bx, by, bz};
    const int cc[3] = {x, y, z};
    float pl[3][4], ph[3][4], pb[3], pa[3], pk[3], pdk[3], zo[3];
    float *zp[3];
    bool slab[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int k = cc[d], n = coord_n(s, d);
        slab[d] = band[d] && in_slab(k, n, s.Llo[d], s.Lhi[d]);
        zp[d] = nullptr;
        zo[d] = 0.0f;
        pb[d] = pa[d] = pk[d] = pdk[d] = 0.0f;
#pragma unroll
        for (int l = 0; l < 4; ++l) pl[d][l] = ph[d][l] = 0.0f;
        if (band[d]) {
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                pl[d][l - 1] = psi_at(s, d, x - (d == 0) * l, y - (d == 1) * l, z - (d == 2) * l);
                ph[d][l - 1] = psi_at(s, d, x + (d == 0) * l, y + (d == 1) * l, z + (d == 2) * l);
            }
            pb[d] = prof_at(s, d, 0, k);
            pa[d] = prof_at(s, d, 1, k);
            pk[d] = prof_at(s, d, 2, k);
            pdk[d] = prof_at(s, d, 3, k);
            if (slab[d]) {
                zp[d] = &s.zeta[d][psi_index(s, d, x, y, z)];
                zo[d] = *zp[d];
            }
        }
    }
    float L[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float d2 = d2_axis(s.w2[d], c, lo[d], hi[d]);
        if (!band[d]) {
            L[d] = d2;
            continue;
        }
        const float d1 = d1_axis(s.w1[d], lo[d], hi[d]);
        const float dpsi = d1_axis(s.w1[d], pl[d], ph[d]);
        float zn = 0.0f;
        L[d] = cpml_axis(d2, d1, dpsi, pk[d], pdk[d], pa[d], pb[d], slab[d], zo[d], &zn);
        if (slab[d]) *zp[d] = zn;
    }
    return (L[0] + L[1]) + L[2];
}

// source amplitude (already multiplied by storage scale / cell volume) at step n
__device__ __forceinline__ float source_at(const DevShot &s, int n) {
    return (s.wav != nullptr && n >= 0 && n < s.src_nt) ? s.wav[n] * s.src_scale : 0.0f;
}

// coordinate folded back into [0, n) on a ghost (periodic loopback) axis
__device__ __forceinline__ int wrap_ghost(const DevShot &s, int d, int c) {
    const int n = coord_n(s, d);
    if (s.ghost[d]) {
        if (c < 0) c += n;
        else if (c >= n) c -= n;
    }
    return c;
}
// the source node, or one of its periodic images in the ghost rows/planes
__device__ __forceinline__ bool is_source(const DevShot &s, int x, int y, int z) {
    return x == s.sx && wrap_ghost(s, 1, y) == s.sy && wrap_ghost(s, 2, z) == s.sz;
}

__device__ __forceinline__ bool any_band(const DevShot &s, int x, int y, int z) {
    return in_band(x, s.nx, s.Llo[0], s.Lhi[0]) || in_band(y, s.ny, s.Llo[1], s.Lhi[1]) ||
           in_band(z, s.nz, s.Llo[2], s.Lhi[2]);
}

// Time update of one point.  FP32 storage keeps (u^n, u^{n-1}) and writes
// u^{n+1} = leapfrog(m, Lt, u^n, u^{n-1}) (+ m src) over u^{n-1}.  16-bit
// storage keeps (u^n, d^n = u^n - u^{n-1}) and advances the same recurrence as
//   d^{n+1} = d^n + m Lt (+ m src),   u^{n+1} = u^n + d^{n+1},
// rounding d^{n+1} first and forming u^{n+1} from the stored d^{n+1}: a 16-bit
// rounding of u then perturbs the position only, instead of acting as a
// velocity error that the leapfrog amplifies by ~1/(omega dt).
template <typename T> struct IsInc { static constexpr bool v = sizeof(T) == 2; };

struct Upd {
    float u;   // new u (u^{n+1})
    float d;   // new d (16-bit path) -- equals the value stored
};
template <typename T>
__device__ __forceinline__ Upd time_update(float m, float lt, float c, float second, bool add_src, float src) {
    Upd r;
    if constexpr (IsInc<T>::v) {
        float dn = fmaf(m, lt, second);
        if (add_src) dn = fmaf(m, src, dn);
        const float dr = (float)(T)dn;
        r.d = dr;
        r.u = c + dr;
    } else {
        float un = leapfrog(m, lt, c, second);
        if (add_src) un = fmaf(m, src, un);
        r.u = un;
        r.d = 0.0f;
    }
    return r;
}

// Full update of one point with every neighbour read from memory:
// u^{n+1} = leapfrog(m, Lt, u^n, u^{n-1}) (+ m * src at the source node),
// written over u^{n-1}.  The naive kernel uses it for every point and the
// z-marching kernels for the points of the layer bands.
template <typename T>
__device__ __forceinline__ void point_update_global(const DevShot &s, const T *__restrict__ u,
                                                    const T *__restrict__ um, T *__restrict__ w, int x, int y, int z,
                                                    float src) {
    const long c = (long)z * s.S + (long)y * s.P + x;
    float xl[4], xh[4], yl[4], yh[4], zl[4], zh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        xl[l - 1] = Store<T>::ld(u + c - l);
        xh[l - 1] = Store<T>::ld(u + c + l);
        yl[l - 1] = Store<T>::ld(u + c - (long)l * s.P);
        yh[l - 1] = Store<T>::ld(u + c + (long)l * s.P);
        zl[l - 1] = Store<T>::ld(u + c - (long)l * s.S);
        zh[l - 1] = Store<T>::ld(u + c + (long)l * s.S);
    }
    const float uc = Store<T>::ld(u + c);
    const float mm = s.m[c];
    T *sec = IsInc<T>::v ? (T *)s.dinc : (T *)um;
    const float second = Store<T>::ld(sec + c);
    const float lt = lap_point(s, x, y, z, uc, xl, xh, yl, yh, zl, zh);
    const Upd r = time_update<T>(mm, lt, uc, second, is_source(s, x, y, z), src);
    Store<T>::st(w + c, r.u);
    if constexpr (IsInc<T>::v) Store<T>::st(sec + c, r.d);
}
