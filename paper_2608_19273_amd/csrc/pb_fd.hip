// pb_fd.hip -- one Runge-Kutta stage of the fourth-order finite-difference
// scheme with sixth-order Kreiss-Oliger dissipation for the linear symmetric
// system dQ/dt + sum_d B_d dQ/dx_d = 0 on independent periodic patches:
//   R(Q) = sum_d ( -B_d D4_d Q + KO6_d Q ),
//   D4 u  = [(u_-2 - u_+2) + 8 (u_+1 - u_-1)] / (12 dx),
//   KO6 u = sigma/(64 dx) [(u_-3 + u_+3) - 6 (u_-2 + u_+2) + 15 (u_-1 + u_+1) - 20 u_0].
//
// Two kernels compute the same stage with the same arithmetic in the same
// order (bitwise equal results): fd_stage_kernel below, in which every wave
// runs every phase, and fd_stage_ws_kernel further down (the default), which
// splits the phases between producer and consumer waves.
//
// Work decomposition of fd_stage_kernel (MI355X): one persistent launch per
// RK stage, two work-groups of four waves per CU.  Work items are 4x4x4 cell tiles, listed
// largest patches first with the tiles of a patch consecutive; the launch
// walks the list in rounds of gridDim.x items, and inside a round the
// work-groups of one XCD take one contiguous run (one whole 16^3 patch), so a
// patch is fetched into that XCD's L2 once.  For a tile, the N unknowns are
// processed in chunks of 8:
//   1. the chunk's values on the tile's stencil footprint are copied from HBM
//      straight into LDS by the gfx950 global->LDS DMA loads (16 bytes = two
//      x-adjacent cells per lane, no registers involved).  The footprint of
//      one unknown is 384 doubles: 16 rows of 12 cells along x (the tile's
//      rows with 4 halo cells on each side, one of them unused), and the 3
//      halo layers on the -y, +y, -z, +z faces as rows of 4 cells;
//      periodic wrap inside the patch.  The DMA for the next chunk (or the
//      next tile's first chunk) is issued into the other of two buffers
//      before the current chunk is computed, so HBM/L2 latency overlaps the
//      arithmetic;
//   2. every (unknown, cell) pair of the chunk gets D4_x, D4_y, D4_z (the
//      gradient G_d, stored in LDS as matrix-core operands) and the summed
//      KO6 term.  A thread always owns the same cell, so its 13 stencil
//      addresses are computed once per launch;
//   3. the dense product -sum_d B_d G_d runs on the FP64 matrix cores
//      (v_mfma_f64_16x16x4f64): wave w owns output rows 16w..16w+15 and keeps
//      its rows of -B_d (K padded to 60) in registers for the whole launch,
//      accumulating over chunks and directions;
// then the stage update (RK4 Butcher weights) is applied in the matrix-core
// output layout.  For v_mfma_f64_16x16x4f64 lane l holds A[l%16][l/16] and
// B[l/16][l%16] and its four result registers i hold D[4i + l/16][l%16]
// (rows step by 4 across registers; checked on the device).
//
// Barriers: the plain work-group barrier also waits for every outstanding
// memory operation of the wave (including the DMA just issued for the next
// chunk), which would serialise the pipeline.  The kernel therefore waits
// explicitly (vmcnt: all but the DMA issued for the next chunk; lgkmcnt: LDS
// writes) and then issues the bare barrier instruction, with a compiler
// memory clobber so no LDS access moves across it.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pb_common.h"

namespace pb {

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
#define PB_LDS(ptr) ((__attribute__((address_space(3))) void *)(ptr))

constexpr int kFdThreads = 256;
constexpr int kT = 4;                  // tile edge
constexpr int kTC = kT * kT * kT;      // 64 cells per tile
constexpr int kCh = 8;                 // unknowns per chunk
constexpr int kMaxCh = 8;              // chunks per tile (N <= 60, rounded up to even)
constexpr int kRowX = 12;              // x-extended row: x in [-4, 8)
constexpr int kRegY = 16 * kRowX;      // 192: first y-halo row
constexpr int kRegZ = kRegY + 24 * kT; // 288: first z-halo row
constexpr int kFoot = kRegZ + 24 * kT; // 384 doubles per unknown
constexpr int kMaxN = 60;              // K of the dense product padded to a multiple of 4

// LDS slot of tile-local (x, y, z), at most one coordinate outside [0, 4)
// (x in [-4, 8), y and z in [-3, 7))
__device__ __forceinline__ int foot_slot(int x, int y, int z)
{
    if (y < 0 || y >= kT) return kRegY + (z * 6 + (y < 0 ? y + 3 : y - 1)) * kT + x;
    if (z < 0 || z >= kT) return kRegZ + (y * 6 + (z < 0 ? z + 3 : z - 1)) * kT + x;
    return (z * kT + y) * kRowX + x + 4;
}

// first cell (x, x + 1 share the piece) of 16-byte piece q of the footprint,
// in LDS order: piece q fills slots 2q and 2q + 1
__device__ __forceinline__ void piece_coord(int q, int &x, int &y, int &z)
{
    if (q < kRegY / 2) {
        const int r = q / 6;
        z = r / kT; y = r % kT; x = -4 + 2 * (q % 6);
    } else if (q < kRegZ / 2) {
        const int qq = q - kRegY / 2, r = qq / 2, yy = r % 6;
        z = r / 6; y = yy < 3 ? yy - 3 : yy + 1; x = 2 * (qq % 2);
    } else {
        const int qq = q - kRegZ / 2, r = qq / 2, zz = r % 6;
        y = r / 6; z = zz < 3 ? zz - 3 : zz + 1; x = 2 * (qq % 2);
    }
}

struct FdItem {
    int patch;
    int tile;
};

// geometry of one tile as this lane needs it for the DMA
struct TileSrc {
    const double *base;   // y + offset of the patch's block
    long long C;          // cells of the patch (unknown stride)
    int fo[3];            // cell offset (< p^3) of this lane's piece in each of the 3 DMA rounds
};

__device__ __forceinline__ TileSrc tile_src(const double *y, long long off, int p, int tile, int N)
{
    TileSrc t;
    const int nt = p / kT;
    t.C = (long long)p * p * p;
    t.base = y + off * N;
    const int tx = kT * (tile % nt), ty = kT * ((tile / nt) % nt), tz = kT * (tile / (nt * nt));
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        int x, yy, z;
        piece_coord(64 * i + l, x, yy, z);
        // tile origin + footprint offset stays within one period of the patch
        int gx = tx + x, gy = ty + yy, gz = tz + z;
        gx += gx < 0 ? p : (gx >= p ? -p : 0);
        gy += gy < 0 ? p : (gy >= p ? -p : 0);
        gz += gz < 0 ? p : (gz >= p ? -p : 0);
        t.fo[i] = (gz * p + gy) * p + gx;
    }
    return t;
}

// DMA of unknowns v0 + 2w, v0 + 2w + 1 (wave w) of one tile into buf;
// returns the number of DMA instructions this wave issued
__device__ __forceinline__ int issue_chunk(double (&buf)[kCh][kFoot], const TileSrc &t, int v0, int N)
{
    const int w = threadIdx.x >> 6;
    int n = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int vl = 2 * w + u, v = v0 + vl;
        if (v < N) {
            const double *src = t.base + (long long)v * t.C;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                __builtin_amdgcn_global_load_lds(src + t.fo[i], PB_LDS(&buf[vl][128 * i]), 16, 0, 0);
            n += 3;
        }
    }
    return n;
}

// wait until this wave has at most `pending` vector-memory operations in
// flight (the DMA just issued for the next chunk) and its LDS writes are
// done, then the work-group barrier
__device__ __forceinline__ void barrier_keep(int pending)
{
    if (pending >= 6) __builtin_amdgcn_s_waitcnt(0x0076);
    else if (pending >= 3) __builtin_amdgcn_s_waitcnt(0x0073);
    else __builtin_amdgcn_s_waitcnt(0x0070);
    __asm__ volatile("s_barrier" ::: "memory");
}

// LDS writes done, then the work-group barrier
__device__ __forceinline__ void barrier_lds()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __asm__ volatile("s_barrier" ::: "memory");
}

}  // namespace

// stage: 0..3 (RK4) with rk = 4, or 0 with rk = 1
__global__ __launch_bounds__(kFdThreads, 2) void fd_stage_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const PatchDev *__restrict__ patches, const FdItem *__restrict__ items, int n_items,
    const double *__restrict__ Bmat, int N, int stage, int rk, double dt, double sigma, int remap)
{
    __shared__ double sQ0[kCh][kFoot], sQ1[kCh][kFoot];
    __shared__ double sG[3][kCh][kTC];
    __shared__ double sK[kCh][kTC];

    const int t = threadIdx.x, w = t >> 6, l = t & 63, lg = l >> 4, lj = l & 15;
    // rows 16w + lj of -B_d, columns 4 ks + lg: this lane's A operands
    double a[3][kMaxN / 4];
    {
        const int m = 16 * w + lj;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int ks = 0; ks < kMaxN / 4; ++ks) {
                const int k = 4 * ks + lg;
                a[d][ks] = (m < N && k < N) ? -Bmat[(long long)d * N * N + (long long)m * N + k] : 0.0;
            }
    }
    // chunks per tile, even so that every tile starts in buffer 0
    const int nch = (((N + kCh - 1) / kCh) + 1) & ~1;
    // this thread's cell of the gradient phase (the same in every chunk) and
    // its stencil slots
    const int cx = l % kT, cy = (l / kT) % kT, cz = l / (kT * kT);
    const int sc = foot_slot(cx, cy, cz);
    int sy[6], sz[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sy[k] = foot_slot(cx, cy - 3 + k, cz);
        sy[3 + k] = foot_slot(cx, cy + 1 + k, cz);
        sz[k] = foot_slot(cx, cy, cz - 3 + k);
        sz[3 + k] = foot_slot(cx, cy, cz + 1 + k);
    }

    const int G = (int)gridDim.x, slot = remap ? xcd_remap((int)blockIdx.x, G) : (int)blockIdx.x;
    int it = slot;
    if (it >= n_items) return;
    // current tile: patch block offset, edge, 1/dx, tile index, DMA sources
    long long off;
    int p, tile;
    double inv_dx;
    TileSrc src;
    {
        const FdItem item = items[it];
        const PatchDev P = patches[item.patch];
        off = P.off; p = P.p; inv_dx = P.inv_dx; tile = item.tile;
        src = tile_src(y, off, p, tile, N);
    }
    issue_chunk(sQ0, src, 0, N);

    while (true) {
        const int ntile = p / kT;
        const long long C = src.C;
        const int tx = kT * (tile % ntile), ty = kT * ((tile / ntile) % ntile), tz = kT * (tile / (ntile * ntile));
        const double c4 = inv_dx / 12.0, cko = sigma * inv_dx / 64.0;
        // the next tile of this work-group (its first chunk is prefetched
        // during the last chunk of this one)
        const int itn = it + G;
        const bool has_next = itn < n_items;
        long long offn = off;
        int pn = p, tilen = tile;
        double inv_dxn = inv_dx;
        TileSrc srcn = src;
        if (has_next) {
            const FdItem item = items[itn];
            const PatchDev P = patches[item.patch];
            offn = P.off; pn = P.p; inv_dxn = P.inv_dx; tilen = item.tile;
            srcn = tile_src(y, offn, pn, tilen, N);
        }
        f64x4_t accm[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) accm[nt] = (f64x4_t){0.0, 0.0, 0.0, 0.0};

#pragma unroll
        for (int ch = 0; ch < kMaxCh; ++ch) {
            if (ch >= nch) break;
            double (&buf)[kCh][kFoot] = (ch & 1) ? sQ1 : sQ0;
            double (&nbuf)[kCh][kFoot] = (ch & 1) ? sQ0 : sQ1;
            const int v0 = ch * kCh;
            // 1. prefetch the next chunk, then wait for this one
            int pend = 0;
            if (ch + 1 < nch) {
                pend = issue_chunk(nbuf, src, v0 + kCh, N);
            } else if (has_next) {
                pend = issue_chunk(nbuf, srcn, 0, N);
            }
            barrier_keep(pend);
            // 2. gradients and dissipation of the chunk (cell l, unknowns w, w + 4)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int vl = w + 4 * j;
                double g0 = 0.0, g1 = 0.0, g2 = 0.0, ko = 0.0;
                if (v0 + vl < N) {
                    const double *u = buf[vl];
                    const double u0 = u[sc];
                    {
                        const double m3 = u[sc - 3], m2 = u[sc - 2], m1 = u[sc - 1], p1 = u[sc + 1], p2 = u[sc + 2],
                                     p3 = u[sc + 3];
                        g0 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                        ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                    }
                    {
                        const double m3 = u[sy[0]], m2 = u[sy[1]], m1 = u[sy[2]], p1 = u[sy[3]], p2 = u[sy[4]],
                                     p3 = u[sy[5]];
                        g1 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                        ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                    }
                    {
                        const double m3 = u[sz[0]], m2 = u[sz[1]], m1 = u[sz[2]], p1 = u[sz[3]], p2 = u[sz[4]],
                                     p3 = u[sz[5]];
                        g2 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                        ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                    }
                }
                sG[0][vl][l] = g0;
                sG[1][vl][l] = g1;
                sG[2][vl][l] = g2;
                sK[vl][l] = cko * ko;
            }
            barrier_lds();
            // 3. accumulate -B_d G_d over the chunk's K rows on the matrix cores
            if (v0 < N) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int kk = 0; kk < kCh / 4; ++kk) {
                        const int ks = ch * (kCh / 4) + kk;
                        if (ks >= kMaxN / 4) break;
                        const double aop = a[d][ks];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt)
                            accm[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, sG[d][4 * kk + lg][nt * 16 + lj],
                                                                            accm[nt], 0, 0, 0);
                    }
                // the wave whose output rows are this chunk's unknowns adds KO6
                if (w == ch / 2) {
                    const int h = ch % 2;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int ii = 0; ii < 2; ++ii) accm[nt][2 * h + ii] += sK[lg + 4 * ii][nt * 16 + lj];
                }
            }
        }
        // 4. stage update in the output layout, in two rounds of two column
        //    tiles: all reads of a round first (one memory round trip), then
        //    the arithmetic and the stores
        {
            const bool need_q0 = rk == 1 || stage < 3, need_acc = rk == 4 && stage > 0;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                long long gbase[2];
                double q0v[2][4], accv[2][4];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = (2 * half + h) * 16 + lj;
                    const int x = c % kT, yy = (c / kT) % kT, z = c / (kT * kT);
                    gbase[h] = off * N + ((long long)(tz + z) * p + (ty + yy)) * p + (tx + x);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * w + lg + 4 * i;
                        const long long g = gbase[h] + (long long)(r < N ? r : 0) * C;
                        q0v[h][i] = (r < N && need_q0) ? q0[g] : 0.0;
                        accv[h][i] = (r < N && need_acc) ? acc[g] : 0.0;
                    }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * w + lg + 4 * i;
                        if (r >= N) continue;
                        const long long g = gbase[h] + (long long)r * C;
                        const double R = accm[2 * half + h][i];
                        if (rk == 1) {
                            acc[g] = q0v[h][i] + dt * R;
                        } else if (stage == 0) {
                            ynext[g] = q0v[h][i] + 0.5 * dt * R;
                            acc[g] = q0v[h][i] + (dt / 6.0) * R;
                        } else if (stage == 1) {
                            ynext[g] = q0v[h][i] + 0.5 * dt * R;
                            acc[g] = accv[h][i] + (dt / 3.0) * R;
                        } else if (stage == 2) {
                            ynext[g] = q0v[h][i] + dt * R;
                            acc[g] = accv[h][i] + (dt / 3.0) * R;
                        } else {
                            acc[g] = accv[h][i] + (dt / 6.0) * R;
                        }
                    }
            }
        }
        if (!has_next) break;
        it = itn;
        off = offn; p = pn; inv_dx = inv_dxn; tile = tilen;
        src = srcn;
    }
}

// ------------------------------------------------ wave-specialised stage --
//
// The same stage with the phases split between the waves of one 768-thread
// work-group per CU (3 waves per SIMD): waves 0..3 (consumers) hold their
// rows of -B_d in registers and run only the dense product and the stage
// update; waves 4..11 (producers) move data and compute the gradients.  Both
// roles advance in lock step over the same sequence of (tile, chunk) steps,
// one work-group barrier per step (R = chunks per tile + 1 is the size of
// the operand ring below):
//   producers, step s: gradients and dissipation of chunk s + 1 (LDS slot
//     (s+1) % 2); footprint of chunk s + 2 into LDS from registers, then the
//     global loads of chunk s + 4 into those registers; the stage results
//     held in the ring slot of chunk s + 1 (those of chunk s + 1 - R) out to
//     HBM, then the stage-update operands (Q^0 and accumulator rows) of
//     chunk s + 1 into that slot from registers, then the loads of chunk
//     s + 3;
//   consumers, step s: matrix-core product of chunk s (slot s % 2) and, at
//     the last chunk of a tile, the stage update from the LDS operand ring,
//     whose results replace the operands in the ring (no consumer touches
//     HBM after the start).
// Every copy goes HBM/L2 -> registers -> LDS with ordinary loads issued two
// steps before the data is needed, so the compiler tracks each load by its
// registers and the copies overlap the arithmetic.  The operand ring has one
// slot more than a tile has chunks: a slot is written one step before its
// chunk, read and overwritten with the results at the tile's last step, and
// its results go out to HBM right before it is refilled, at least one step
// later (those of the last tile after the last step).
// Indexes past the last step are clamped to it (that chunk is loaded,
// written and differentiated again and nobody reads the result), except the
// operand ring, which is not written past the last chunk.
namespace {

constexpr int kWsThreads = 768;

}  // namespace

// one work item of the wave-specialised kernel with its geometry resolved on
// the host (a single 32-byte scalar load per tile)
struct alignas(32) WsItem {
    long long off;        // first cell of the patch
    int p, tx, ty, tz;    // patch edge, tile origin
    double inv_dx;
};
static_assert(sizeof(WsItem) == 32, "WsItem layout");

namespace {

// footprint sources of this lane (as tile_src) for a tile given by its origin
__device__ __forceinline__ TileSrc tile_src_at(const double *y, const WsItem &T, int N)
{
    TileSrc t;
    const int p = T.p;
    t.C = (long long)p * p * p;
    t.base = y + T.off * N;
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        int x, yy, z;
        piece_coord(64 * i + l, x, yy, z);
        int gx = T.tx + x, gy = T.ty + yy, gz = T.tz + z;
        gx += gx < 0 ? p : (gx >= p ? -p : 0);
        gy += gy < 0 ? p : (gy >= p ? -p : 0);
        gz += gz < 0 ? p : (gz >= p ? -p : 0);
        t.fo[i] = (gz * p + gy) * p + gx;
    }
    return t;
}

typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <int NCH>
struct WsLds {
    static constexpr int R = NCH + 1;    // operand ring slots
    double q[2][kCh][kFoot];             // footprint ring
    double g[2][3][kCh][kTC];            // gradients (matrix-core B operands)
    double k[2][kCh][kTC];               // summed dissipation
    double u[R][2][kCh][kTC];            // update operands: [slot][Q^0-side, acc-side][unknown][cell]
};

// producer waves: footprints, gradients and dissipation, update operands
template <int NCH>
__device__ __forceinline__ void ws_producer(WsLds<NCH> &L, const double *__restrict__ y,
                                            const double *__restrict__ srcq, const double *__restrict__ srca,
                                            double *__restrict__ acc, double *__restrict__ ynext, bool write_y,
                                            const WsItem *__restrict__ items, int slot, int G, int S, int N,
                                            double sigma)
{
    constexpr int R = WsLds<NCH>::R;
    // pw (the producer wave) is the same in every lane: as a scalar, the
    // chunk's unknown and every offset derived from it stay on the scalar
    // unit instead of costing 64-bit vector multiplies per step
    const int t = threadIdx.x - 256, pw = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63;
    const int cx = l % kT, cy = (l / kT) % kT, cz = l / (kT * kT);
    const int sc = foot_slot(cx, cy, cz);
    int sy[6], sz[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sy[k] = foot_slot(cx, cy - 3 + k, cz);
        sy[3 + k] = foot_slot(cx, cy + 1 + k, cz);
        sz[k] = foot_slot(cx, cy, cz - 3 + k);
        sz[3 + k] = foot_slot(cx, cy, cz + 1 + k);
    }
    // this thread's piece of the update operands of a chunk: side (Q^0 or
    // accumulator), unknown within the chunk, two x-adjacent cells
    const int us = t >> 8, uv = (t >> 5) & 7, uc = 2 * (t & 31);
    const int ux = uc % kT, uy = (uc / kT) % kT, uz = uc / (kT * kT);
    const double *__restrict__ usrc = us ? srca : srcq;
    // tile caches of the three cursors (footprint loads, gradients, operand loads)
    int kf = -1, kg = -1, ku = -1, ko = -1;
    TileSrc fsrc{};
    double inv_dx = 0.0;
    long long ubase = 0, uC = 0, obase = 0, oC = 0;

    auto load_foot = [&](int c, f64x2_t (&F)[3]) {
        c = c < S ? c : S - 1;
        const int k = c / NCH, ch = c - k * NCH;
        if (k != kf) {
            kf = k;
            fsrc = tile_src_at(y, items[slot + k * G], N);
        }
        const int v0 = ch * kCh + pw, v = v0 < N ? v0 : N - 1;
        const double *s = fsrc.base + (long long)v * fsrc.C;
#pragma unroll
        for (int i = 0; i < 3; ++i) F[i] = *reinterpret_cast<const f64x2_t *>(s + fsrc.fo[i]);
    };
    auto stage_foot = [&](int b, const f64x2_t (&F)[3]) {
#pragma unroll
        for (int i = 0; i < 3; ++i) *reinterpret_cast<f64x2_t *>(&L.q[b][pw][128 * i + 2 * l]) = F[i];
    };
    auto load_upd = [&](int c) -> f64x2_t {
        c = c < S ? c : S - 1;
        const int k = c / NCH, ch = c - k * NCH;
        if (k != ku) {
            ku = k;
            const WsItem T = items[slot + k * G];
            const int p = T.p;
            uC = (long long)p * p * p;
            ubase = T.off * N + ((long long)(T.tz + uz) * p + (T.ty + uy)) * p + (T.tx + ux);
        }
        const int v0 = ch * kCh + uv, v = v0 < N ? v0 : N - 1;
        // v < 64 and uC = p^3 <= 4096: a 24-bit product
        return *reinterpret_cast<const f64x2_t *>(usrc + ubase + __umul24((unsigned)v, (unsigned)uC));
    };
    auto stage_upd = [&](int c, const f64x2_t &U) {
        if (c < S) *reinterpret_cast<f64x2_t *>(&L.u[c % R][us][uv][uc]) = U;
    };
    // the stage results of chunk c (written into its ring slot by the
    // consumers at the tile's last step) to HBM: new accumulator (side 0)
    // and next stage value (side 1, where the stage has one)
    auto store_out = [&](int c) {
        if (c < 0) return;
        const int k = c / NCH, ch = c - k * NCH;
        if (k != ko) {
            ko = k;
            const WsItem T = items[slot + k * G];
            const int p = T.p;
            oC = (long long)p * p * p;
            obase = T.off * N + ((long long)(T.tz + uz) * p + (T.ty + uy)) * p + (T.tx + ux);
        }
        const int v = ch * kCh + uv;
        if (v < N && (us == 0 || write_y)) {
            const f64x2_t r = *reinterpret_cast<const f64x2_t *>(&L.u[c % R][us][uv][uc]);
            double *dst = us ? ynext : acc;
            *reinterpret_cast<f64x2_t *>(dst + obase + __umul24((unsigned)v, (unsigned)oC)) = r;
        }
    };
    auto grad = [&](int c) {
        c = c < S ? c : S - 1;
        const int k = c / NCH, ch = c - k * NCH, b = c & 1;
        if (k != kg) {
            kg = k;
            inv_dx = items[slot + k * G].inv_dx;
        }
        const double c4 = inv_dx / 12.0, cko = sigma * inv_dx / 64.0;
        const int vl = pw;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, ko = 0.0;
        if (ch * kCh + vl < N) {
            const double *u = L.q[b][vl];
            const double u0 = u[sc];
            {
                const double m3 = u[sc - 3], m2 = u[sc - 2], m1 = u[sc - 1], p1 = u[sc + 1], p2 = u[sc + 2],
                             p3 = u[sc + 3];
                g0 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
            }
            {
                const double m3 = u[sy[0]], m2 = u[sy[1]], m1 = u[sy[2]], p1 = u[sy[3]], p2 = u[sy[4]],
                             p3 = u[sy[5]];
                g1 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
            }
            {
                const double m3 = u[sz[0]], m2 = u[sz[1]], m1 = u[sz[2]], p1 = u[sz[3]], p2 = u[sz[4]],
                             p3 = u[sz[5]];
                g2 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
            }
        }
        L.g[b][0][vl][l] = g0;
        L.g[b][1][vl][l] = g1;
        L.g[b][2][vl][l] = g2;
        L.k[b][vl][l] = cko * ko;
    };

    // step -2 and -1 (before the consumers' first product), then steps 0..S-1;
    // footprint sets: FA for even steps, FB for odd; operand sets: UB for
    // even steps, UA for odd
    f64x2_t FA[3], FB[3], UA, UB;
    load_foot(0, FA);
    load_foot(1, FB);
    UA = load_upd(0);
    // step -2
    stage_foot(0, FA);
    load_foot(2, FA);
    UB = load_upd(1);
    lds_barrier();
    // step -1
    grad(0);
    stage_foot(1, FB);
    load_foot(3, FB);
    stage_upd(0, UA);
    UA = load_upd(2);
    lds_barrier();
    // each step first writes out the results held in the ring slot it is
    // about to refill (chunk c - R, whose tile ended at least one step ago)
    for (int s = 0; s < S; s += 2) {
        grad(s + 1);
        stage_foot(0, FA);
        load_foot(s + 4, FA);
        store_out(s + 1 - R);
        stage_upd(s + 1, UB);
        UB = load_upd(s + 3);
        lds_barrier();
        if (s + 1 >= S) break;
        grad(s + 2);
        stage_foot(1, FB);
        load_foot(s + 5, FB);
        store_out(s + 2 - R);
        stage_upd(s + 2, UA);
        UA = load_upd(s + 4);
        lds_barrier();
    }
    // the last tile's results (its update ran at the final step, before the
    // last barrier)
    for (int c = S - NCH > 0 ? S - NCH : 0; c < S; ++c) store_out(c);
}

// consumer waves: -sum_d B_d G_d on the matrix cores and the stage update
template <int NCH>
__device__ __forceinline__ void ws_consumer(WsLds<NCH> &L, const WsItem *__restrict__ items, int slot, int G,
                                            int n_my,
                                            const double *__restrict__ Bmat, int N, int stage, int rk, double dt)
{
    constexpr int R = WsLds<NCH>::R;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lg = l >> 4, lj = l & 15;
    double a[3][kMaxN / 4];
    {
        const int m = 16 * w + lj;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int ks = 0; ks < kMaxN / 4; ++ks) {
                // every lane loads (clamped index), so no load sits in a branch
                const int k = 4 * ks + lg;
                const double bv = Bmat[(long long)d * N * N + (long long)(m < N ? m : N - 1) * N + (k < N ? k : N - 1)];
                a[d][ks] = (m < N && k < N) ? -bv : 0.0;
            }
    }
    // the stage update, with one form for every stage:
    //   acc <- (Q^0-side) + ca R,   ynext <- Q^0 + cy R (stages 1-3 of RK4);
    // the operand ring holds Q^0 (or, where a stage needs no Q^0, the
    // accumulator) on one side and the accumulator (or Q^0) on the other
    const bool from_q0 = !(rk == 4 && stage > 0);
    const double ca = rk == 1 ? dt : ((stage == 0 || stage == 3) ? dt / 6.0 : dt / 3.0);
    const double cy = stage == 2 ? dt : 0.5 * dt;
    lds_barrier();
    lds_barrier();
    int s = 0;
    for (int kt = 0; kt < n_my; ++kt) {
        f64x4_t accm[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) accm[nt] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch, ++s) {
            const int b = s & 1;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int kk = 0; kk < kCh / 4; ++kk) {
                    const int ks = ch * (kCh / 4) + kk;
                    if (ks >= kMaxN / 4) break;
                    const double aop = a[d][ks];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        accm[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, L.g[b][d][4 * kk + lg][nt * 16 + lj],
                                                                        accm[nt], 0, 0, 0);
                }
            if (w == ch / 2) {
                const int h = ch % 2;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii) accm[nt][2 * h + ii] += L.k[b][lg + 4 * ii][nt * 16 + lj];
            }
            if (ch == NCH - 1) {
                // element (nt, i) of this lane: unknown r = 16 w + lg + 4 i,
                // cell nt * 16 + lj of the tile.  The results replace the
                // operands in the ring slot (the producers write them to HBM
                // over the next tile's steps); rows at or beyond N are
                // skipped (beyond the last chunk a row would alias one of it)
                double *ul = &L.u[0][0][lg][lj];
                const int c0 = s - ch;   // global index of the tile's first chunk
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // operand ring slot of unknown row r (its chunk is 2 w + i / 2)
                    const int rc = 2 * w + i / 2 < NCH ? 2 * w + i / 2 : NCH - 1;
                    double *ui = ul + ((c0 + rc) % R) * (2 * kCh * kTC) + 4 * (i % 2) * kTC;
                    const bool live = 16 * w + lg + 4 * i < N;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const double R0 = accm[nt][i], qv = ui[nt * 16], av = ui[kCh * kTC + nt * 16];
                        const double an = (from_q0 ? qv : av) + ca * R0, yn = qv + cy * R0;
                        if (live) {
                            ui[nt * 16] = an;
                            ui[kCh * kTC + nt * 16] = yn;
                        }
                    }
                }
            }
            lds_barrier();
        }
    }
}

}  // namespace

template <int NCH>
__global__ __launch_bounds__(kWsThreads) void fd_stage_ws_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const WsItem *__restrict__ items, int n_items, const double *__restrict__ Bmat, int N,
    int stage, int rk, double dt, double sigma, int remap)
{
    __shared__ WsLds<NCH> L;
    const int G = (int)gridDim.x, slot = remap ? xcd_remap((int)blockIdx.x, G) : (int)blockIdx.x;
    if (slot >= n_items) return;
    const int n_my = (n_items - slot + G - 1) / G;
    if (threadIdx.x >= 256) {
        // the stage's update operands: Q^0 and the accumulator where it needs
        // both, else the one it needs on both sides
        const bool need_q0 = rk == 1 || stage < 3, need_acc = rk == 4 && stage > 0;
        ws_producer<NCH>(L, y, need_q0 ? q0 : acc, need_acc ? acc : q0, acc, ynext, rk == 4 && stage < 3, items,
                         slot, G, n_my * NCH, N, sigma);
    } else {
        ws_consumer<NCH>(L, items, slot, G, n_my, Bmat, N, stage, rk, dt);
    }
}

// ------------------------------------------------ one wave per tile --
//
// fd_ws = 2: every wave advances whole 4x4x4 tiles on its own, with no
// work-group barrier.  Per chunk of four unknowns (one K step of the matrix
// product):
//   1. the chunk's footprints (4 x 384 doubles) and its A operands (rows of
//      -B_d for the four unknowns, 12 x 64 doubles of a packed table, L2-
//      resident) go HBM/L2 -> the wave's own LDS by the global->LDS DMA, one
//      chunk ahead, double buffered (no register holds data in flight, and
//      every memory instruction of the chunk loop is one of these copies, so
//      the wait for a chunk is an exact count);
//   2. lane l differentiates unknown 4c + l/16 at the tile cells 16 nt + l%16
//      (nt = 0..3, the tile's z planes): its D4_d values are exactly the B
//      operands of v_mfma_f64_16x16x4f64 for column tile nt, and its KO6 value
//      sits in the same lane and register as the accumulator of that row and
//      cell, so nothing is transposed;
//   3. 48 matrix instructions (3 directions x 4 row tiles x 4 column tiles)
//      accumulate -sum_d B_d G_d for 64 rows x 64 cells in registers, then the
//      chunk's KO6 is added to its rows.
// After the last chunk the stage update runs in the matrix-core output layout
// (lane l, register i of tile (rt, nt): row 16 rt + 4 i + l/16, cell
// 16 nt + l%16).  The arithmetic is the other stage kernels' formula by
// formula; only the order of the additions over the K steps differs (four
// unknowns per step, directions in order), so results agree to roundoff.
constexpr int kTileCh = 4;                   // unknowns per chunk (one K step)
constexpr int kTileMaxCh = kMaxN / kTileCh;  // 15 chunks for N <= 60
constexpr int kTileA = 3 * 4 * 64;           // A operands of one chunk (doubles)
constexpr int kTileDma = kTileCh * 3 + kTileA / 128;   // copies per chunk: 12 + 6

// this wave's LDS: two chunk buffers of footprints and A operands
struct TileLds {
    double foot[2][kTileCh][kFoot];
    double a[2][kTileA];
};

// one chunk's copies (unknowns >= N are read from unknown N - 1: their
// gradients are zeroed, and their A columns are zero)
__device__ __forceinline__ void tile_dma(TileLds &L, int buf, const TileSrc &t, const double *apk, int c, int N)
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < kTileCh; ++u) {
        const int v = min(c * kTileCh + u, N - 1);
        const double *src = t.base + (long long)v * t.C;
#pragma unroll
        for (int i = 0; i < 3; ++i) dma_to_lds16(src + t.fo[i], &L.foot[buf][u][128 * i]);
    }
    const double *as = apk + (long long)c * kTileA + 2 * l;
#pragma unroll
    for (int i = 0; i < kTileA / 128; ++i) dma_to_lds16(as + 128 * i, &L.a[buf][128 * i]);
}

// wait until at most 18 (the next chunk's copies) / 0 of this wave's vector
// memory operations are in flight, leaving the LDS counter unconstrained;
// the empty asm keeps LDS reads of the chunk after the wait
__device__ __forceinline__ void tile_wait_next()
{
    static_assert(kTileDma == 18, "vmcnt immediate below");
    __builtin_amdgcn_s_waitcnt(0x4F72);   // vmcnt(18) = [3:0] 2, [15:14] 1; expcnt 7; lgkmcnt 15
    __asm__ volatile("" ::: "memory");
}
__device__ __forceinline__ void tile_wait_all()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt 7, lgkmcnt 15
    __asm__ volatile("" ::: "memory");
}

__global__ __launch_bounds__(64) void fd_stage_tile_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const WsItem *__restrict__ items, int n_items, const double *__restrict__ apk,
    int N, int stage, int rk, double dt, double sigma, int remap)
{
    __shared__ TileLds L;
    const int l = threadIdx.x, g = l >> 4, j = l & 15;
    const int x = j & 3, yy = j >> 2;
    const int G = (int)gridDim.x, slot = remap ? xcd_remap((int)blockIdx.x, G) : (int)blockIdx.x;
    const int nch = (N + kTileCh - 1) / kTileCh;
    // footprint slots of the lane's column (x, yy) (see foot_slot): plane z
    // of the tile at 48 z + ib; a y neighbour at offset k at ysl[k] + z ystr[k];
    // a z neighbour in halo layer h (0..5) at zb + 4 h
    const int ib = yy * 12 + x + 4;
    const int zb = kRegZ + yy * 24 + x;
    int ysl[6], ystr[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int yo = k < 3 ? yy - 3 + k : yy + k - 2;   // yy-3..yy-1, yy+1..yy+3
        if (yo >= 0 && yo < kT) {
            ysl[k] = yo * 12 + x + 4;
            ystr[k] = 48;
        } else {
            ysl[k] = kRegY + (yo < 0 ? yo + 3 : yo - 1) * kT + x;
            ystr[k] = 24;
        }
    }
    const bool need_q0 = rk == 1 || stage < 3, need_acc = rk == 4 && stage > 0;
    int buf = 0;
    for (int it = slot; it < n_items; it += G) {
        const WsItem W = items[it];
        const int p = W.p, ntl = p / kT;
        const TileSrc src = tile_src(y, W.off, p, ((W.tz / kT) * ntl + W.ty / kT) * ntl + W.tx / kT, N);
        const double c4 = W.inv_dx / 12.0, cko = sigma * W.inv_dx / 64.0;
        f64x4_t am[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) am[rt][nt] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
        tile_dma(L, buf, src, apk, 0, N);
        // fully unrolled: the KO6 rows of chunk c are a fixed accumulator register
#pragma clang loop unroll(full)
        for (int c = 0; c < kTileMaxCh; ++c) {
            if (c >= nch) continue;   // (not break: a constant trip count lets the loop unroll)
            // keep each chunk's instructions together: scheduling across the
            // unrolled chunks would hold several chunks' values at once
            __builtin_amdgcn_sched_barrier(0);
            const int cur = buf;
            if (c + 1 < nch) {
                buf ^= 1;
                // the chunk index as a value the compiler cannot see through:
                // otherwise it computes every chunk's copy addresses up front
                int cn = c + 1, bn = buf;
                __asm__ volatile("" : "+s"(cn), "+s"(bn));
                tile_dma(L, bn, src, apk, cn, N);
                tile_wait_next();
            } else {
                tile_wait_all();
            }
            // gradients and dissipation of unknown 4c + g at the lane's cells
            const bool live = c * kTileCh + g < N;
            const double *uf = L.foot[cur][g];
            double gd[3][4], ko[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int sc = 48 * nt + ib;
                const double u0 = uf[sc];
                double g0, g1, g2, k;
                {
                    const double m3 = uf[sc - 3], m2 = uf[sc - 2], m1 = uf[sc - 1], p1 = uf[sc + 1], p2 = uf[sc + 2],
                                 p3 = uf[sc + 3];
                    g0 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    k = ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                {
                    const double m3 = uf[ysl[0] + nt * ystr[0]], m2 = uf[ysl[1] + nt * ystr[1]],
                                 m1 = uf[ysl[2] + nt * ystr[2]], p1 = uf[ysl[3] + nt * ystr[3]],
                                 p2 = uf[ysl[4] + nt * ystr[4]], p3 = uf[ysl[5] + nt * ystr[5]];
                    g1 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    k += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                {
                    // z neighbours nt-3..nt+3: a plane of the tile or a halo layer
                    auto zs = [&](int z) { return z >= 0 && z < kT ? 48 * z + ib : zb + 4 * (z < 0 ? z + 3 : z - 1); };
                    const double m3 = uf[zs(nt - 3)], m2 = uf[zs(nt - 2)], m1 = uf[zs(nt - 1)], p1 = uf[zs(nt + 1)],
                                 p2 = uf[zs(nt + 2)], p3 = uf[zs(nt + 3)];
                    g2 = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    k += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                gd[0][nt] = live ? g0 : 0.0;
                gd[1][nt] = live ? g1 : 0.0;
                gd[2][nt] = live ? g2 : 0.0;
                ko[nt] = live ? cko * k : 0.0;
            }
            // -sum_d B_d G_d over this K step (A operands from this chunk's LDS copy)
            const double *ap = &L.a[cur][l];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const double a = ap[(d * 4 + rt) * 64];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        am[rt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, gd[d][nt], am[rt][nt], 0, 0, 0);
                }
            // KO6 of unknown 4c + g: row 16 (c/4) + 4 (c%4) + g of the output layout
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) am[c / 4][nt][c % 4] += ko[nt];
        }
        buf ^= 1;   // the next tile's first chunk goes to the other buffer
        // stage update, one row tile at a time (all loads of a round first)
        const long long C = (long long)p * p * p, pp = (long long)p * p;
        const long long cell = ((long long)W.tz * p + (W.ty + yy)) * p + (W.tx + x);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            double qv[4][4], av[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + 4 * i + g;
                const long long gr = W.off * N + (long long)(r < N ? r : 0) * C + cell;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    qv[i][nt] = (r < N && need_q0) ? q0[gr + nt * pp] : 0.0;
                    av[i][nt] = (r < N && need_acc) ? acc[gr + nt * pp] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + 4 * i + g;
                if (r >= N) continue;
                const long long gr = W.off * N + (long long)r * C + cell;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const long long gi = gr + nt * pp;
                    const double R = am[rt][nt][i];
                    if (rk == 1) {
                        acc[gi] = qv[i][nt] + dt * R;
                    } else if (stage == 0) {
                        ynext[gi] = qv[i][nt] + 0.5 * dt * R;
                        acc[gi] = qv[i][nt] + (dt / 6.0) * R;
                    } else if (stage == 1) {
                        ynext[gi] = qv[i][nt] + 0.5 * dt * R;
                        acc[gi] = av[i][nt] + (dt / 3.0) * R;
                    } else if (stage == 2) {
                        ynext[gi] = qv[i][nt] + dt * R;
                        acc[gi] = av[i][nt] + (dt / 3.0) * R;
                    } else {
                        acc[gi] = av[i][nt] + (dt / 6.0) * R;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host --

pb_status fd_prepare(pb_batch *b)
{
    if (b->fd_ready) return PB_OK;
    std::vector<FdItem> items;
    // largest patches first (cost ~ p^3), tiles of one patch consecutive
    std::vector<int> order((size_t)b->K);
    for (int k = 0; k < b->K; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->p[x] > b->p[y]; });
    for (int k : order) {
        const int nt = b->p[k] / kT;
        for (int t = 0; t < nt * nt * nt; ++t) items.push_back({k, t});
    }
    const size_t nB = (size_t)3 * b->N * b->N;
    std::vector<WsItem> ws((size_t)items.size());
    {
        std::vector<long long> off((size_t)b->K + 1, 0);
        for (int k = 0; k < b->K; ++k) off[k + 1] = off[k] + (long long)b->p[k] * b->p[k] * b->p[k];
        for (size_t i = 0; i < items.size(); ++i) {
            const int k = items[i].patch, p = b->p[k], nt = p / kT, t = items[i].tile;
            ws[i] = WsItem{off[k], p, kT * (t % nt), kT * ((t / nt) % nt), kT * (t / (nt * nt)), 1.0 / b->dx[k]};
        }
    }
    PB_HIP(hipMalloc(&b->d_fd_ws_items, ws.size() * sizeof(WsItem)));
    PB_HIP(hipMemcpy(b->d_fd_ws_items, ws.data(), ws.size() * sizeof(WsItem), hipMemcpyHostToDevice));
    // A operands of the one-wave-per-tile kernel: per chunk c of four
    // unknowns, direction d, row tile rt and lane l, -B_d[16 rt + l%16][4 c + l/16]
    // (zero outside N x N)
    {
        const int N = b->N;
        std::vector<double> apk((size_t)kTileMaxCh * kTileA, 0.0);
        for (int c = 0; c < kTileMaxCh; ++c)
            for (int d = 0; d < 3; ++d)
                for (int rt = 0; rt < 4; ++rt)
                    for (int l = 0; l < 64; ++l) {
                        const int r = 16 * rt + l % 16, k = 4 * c + l / 16;
                        if (r < N && k < N)
                            apk[(size_t)c * kTileA + (d * 4 + rt) * 64 + l] =
                                -b->params[3 + (size_t)d * N * N + (size_t)r * N + k];
                    }
        PB_HIP(hipMalloc(&b->d_fd_A, apk.size() * sizeof(double)));
        PB_HIP(hipMemcpy(b->d_fd_A, apk.data(), apk.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    PB_HIP(hipMalloc(&b->d_fd_items, items.size() * sizeof(FdItem)));
    PB_HIP(hipMalloc(&b->d_fd_B, nB * sizeof(double)));
    PB_HIP(hipMemcpy(b->d_fd_items, items.data(), items.size() * sizeof(FdItem), hipMemcpyHostToDevice));
    PB_HIP(hipMemcpy(b->d_fd_B, b->params.data() + 3, nB * sizeof(double), hipMemcpyHostToDevice));
    b->fd_n_items = (int)items.size();
    b->fd_ready = true;
    return PB_OK;
}

pb_status launch_fd_stage(pb_batch *b, int stage, int rk_stages, const void *q0, const void *y, void *ynext,
                          void *acc, double dt, double sigma, hipStream_t s)
{
    pb_status st = fd_prepare(b);
    if (st != PB_OK) return st;
    if (b->N > kMaxN) { set_error("fd_ko_step: at most 60 unknowns"); return PB_EUNSUPPORTED; }
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    int dev = 0, cus = 0;
    PB_HIP(hipGetDevice(&dev));
    PB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (b->fd_ws == 2) {
        // one wave per work-group, as many as the LDS holds (4 per CU)
        const int grid = std::max(1, std::min(b->fd_n_items, cus * 4));
        launch_main(b, fd_stage_tile_kernel, dim3(grid), dim3(64), 0, s, static_cast<const double *>(y),
                    static_cast<const double *>(q0), static_cast<double *>(ynext), static_cast<double *>(acc),
                    reinterpret_cast<const WsItem *>(b->d_fd_ws_items), b->fd_n_items, b->d_fd_A, b->N, stage,
                    rk_stages, dt, sigma, b->fd_xcd_remap);
        PB_HIP(hipGetLastError());
        return PB_OK;
    }
    if (b->fd_ws) {
        // one wave-specialised work-group per CU
        const int grid = std::max(1, std::min(b->fd_n_items, cus));
        const int nch = (b->N + kCh - 1) / kCh;
        auto go = [&](auto kern) {
            launch_main(b, kern, dim3(grid), dim3(kWsThreads), 0, s, static_cast<const double *>(y),
                               static_cast<const double *>(q0), static_cast<double *>(ynext),
                               static_cast<double *>(acc), reinterpret_cast<const WsItem *>(b->d_fd_ws_items),
                               b->fd_n_items, b->d_fd_B, b->N, stage, rk_stages, dt, sigma, b->fd_xcd_remap);
        };
        switch (nch) {
        case 1: go(fd_stage_ws_kernel<1>); break;
        case 2: go(fd_stage_ws_kernel<2>); break;
        case 3: go(fd_stage_ws_kernel<3>); break;
        case 4: go(fd_stage_ws_kernel<4>); break;
        case 5: go(fd_stage_ws_kernel<5>); break;
        case 6: go(fd_stage_ws_kernel<6>); break;
        case 7: go(fd_stage_ws_kernel<7>); break;
        default: go(fd_stage_ws_kernel<8>); break;
        }
        PB_HIP(hipGetLastError());
        return PB_OK;
    }
    const int grid = std::max(1, std::min(b->fd_n_items, cus * b->fd_wg_per_cu));
    launch_main(b, fd_stage_kernel, dim3(grid), dim3(kFdThreads), 0, s, static_cast<const double *>(y),
                       static_cast<const double *>(q0), static_cast<double *>(ynext), static_cast<double *>(acc),
                       b->d_patches, reinterpret_cast<const FdItem *>(b->d_fd_items), b->fd_n_items,
                       b->d_fd_B, b->N, stage, rk_stages, dt, sigma, b->fd_xcd_remap);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

}  // namespace pb
