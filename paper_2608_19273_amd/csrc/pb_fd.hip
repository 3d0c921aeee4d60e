// pb_fd.hip -- one Runge-Kutta stage of the fourth-order finite-difference
// scheme with sixth-order Kreiss-Oliger dissipation for the linear symmetric
// system dQ/dt + sum_d B_d dQ/dx_d = 0 on independent periodic patches:
//   R(Q) = sum_d ( -B_d D4_d Q + KO6_d Q ),
//   D4 u  = [(u_-2 - u_+2) + 8 (u_+1 - u_-1)] / (12 dx),
//   KO6 u = sigma/(64 dx) [(u_-3 + u_+3) - 6 (u_-2 + u_+2) + 15 (u_-1 + u_+1) - 20 u_0].
//
// Work decomposition (MI355X): one persistent launch per RK stage.  Work
// items are 4x4x4 cell tiles, listed largest patches first with the tiles of
// a patch consecutive.  Every tile costs the same, so a static schedule is
// balanced: work-group g takes a contiguous range of the list (neighbouring
// tiles of one patch in sequence, their shared halo cells still in L2) and
// no atomic queue is needed.  For a tile, the N unknowns are processed in
// chunks of 16:
//   1. the chunk's values on the tile's cross-shaped stencil footprint
//      (64 cells + 3 layers on each of the 6 faces = 352 cells, periodic
//      wrap inside the patch) are staged in LDS;
//   2. every (unknown, cell) pair of the chunk gets D4_x, D4_y, D4_z (the
//      gradient G_d, stored in LDS as matrix-core operands) and the summed
//      KO6 term;
//   3. the dense product -sum_d B_d G_d runs on the FP64 matrix cores
//      (v_mfma_f64_16x16x4f64): wave w owns output rows 16w..16w+15 and keeps
//      its rows of -B_d (K padded to 64) in registers for the whole launch,
//      accumulating over chunks and directions;
// then the stage update (RK4 Butcher weights) is applied in the matrix-core
// output layout.  For v_mfma_f64_16x16x4f64 lane l holds A[l%16][l/16] and
// B[l/16][l%16] and its four result registers i hold D[4i + l/16][l%16]
// (rows step by 4 across registers; checked on the device).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pb_common.h"

namespace pb {

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kFdThreads = 256;
constexpr int kT = 4;                 // tile edge
constexpr int kTC = kT * kT * kT;     // 64 cells per tile
constexpr int kCh = 16;               // unknowns per chunk
constexpr int kFoot = kTC + 6 * 3 * kT * kT;  // 352 footprint cells
constexpr int kMaxN = 60;   // K of the dense product padded to a multiple of 4

// footprint slot of tile-local coordinates (x, y, z), at most one of them
// outside [0, 4) and then by at most 3
__device__ __forceinline__ int foot_slot(int x, int y, int z)
{
    if (x < 0) return kTC + 0 * 48 + (x + 3) * 16 + z * 4 + y;
    if (x >= kT) return kTC + 1 * 48 + (x - kT) * 16 + z * 4 + y;
    if (y < 0) return kTC + 2 * 48 + (y + 3) * 16 + z * 4 + x;
    if (y >= kT) return kTC + 3 * 48 + (y - kT) * 16 + z * 4 + x;
    if (z < 0) return kTC + 4 * 48 + (z + 3) * 16 + y * 4 + x;
    if (z >= kT) return kTC + 5 * 48 + (z - kT) * 16 + y * 4 + x;
    return (z * kT + y) * kT + x;
}

// inverse: slot -> tile-local coordinates
__device__ __forceinline__ void foot_coord(int s, int &x, int &y, int &z)
{
    if (s < kTC) {
        x = s % kT; y = (s / kT) % kT; z = s / (kT * kT);
        return;
    }
    const int f = (s - kTC) / 48, r = (s - kTC) % 48, layer = r / 16, a = (r / 4) % 4, b = r % 4;
    switch (f) {
    case 0: x = layer - 3; z = a; y = b; break;
    case 1: x = kT + layer; z = a; y = b; break;
    case 2: y = layer - 3; z = a; x = b; break;
    case 3: y = kT + layer; z = a; x = b; break;
    case 4: z = layer - 3; y = a; x = b; break;
    default: z = kT + layer; y = a; x = b; break;
    }
}

struct FdItem {
    int patch;
    int tile;
};

}  // namespace

// stage: 0..3 (RK4) with rk = 4, or 0 with rk = 1
__global__ __launch_bounds__(kFdThreads, 2) void fd_stage_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const PatchDev *__restrict__ patches, const FdItem *__restrict__ items, int n_items,
    const double *__restrict__ Bmat, int N, int stage, int rk, double dt,
    double sigma, int remap)
{
    __shared__ double sQ[kCh][kFoot];
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
    const int nch = (N + kCh - 1) / kCh;

    // rounds of gridDim.x consecutive items; inside a round the workgroups
    // of one XCD (blockIdx mod 8) take one contiguous run of items, so the
    // tiles of a patch share that XCD's L2 instead of fetching the patch
    // once per XCD
    const int G = (int)gridDim.x, slot = remap ? xcd_remap((int)blockIdx.x, G) : (int)blockIdx.x;
    for (int base = 0; base + slot < n_items; base += G) {
        const FdItem item = items[base + slot];
        const PatchDev P = patches[item.patch];
        const int p = P.p, ntile = p / kT;
        const long long C = (long long)p * p * p;
        const int tx = kT * (item.tile % ntile), ty = kT * ((item.tile / ntile) % ntile),
                  tz = kT * (item.tile / (ntile * ntile));
        const double idx = P.inv_dx;
        const double c4 = idx / 12.0, cko = sigma * idx / 64.0;
        f64x4_t accm[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) accm[nt] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
        // this thread stages footprint slots t and t + 256 (the latter for
        // t < 96); their cell offsets inside the patch are fixed for the tile
        const int s1 = t + kFdThreads;
        const bool has1 = s1 < kFoot;
        long long fo0, fo1 = 0;
        {
            int x, yy, z;
            foot_coord(t, x, yy, z);
            fo0 = ((long long)((tz + z + p) % p) * p + (ty + yy + p) % p) * p + (tx + x + p) % p;
            if (has1) {
                foot_coord(s1, x, yy, z);
                fo1 = ((long long)((tz + z + p) % p) * p + (ty + yy + p) % p) * p + (tx + x + p) % p;
            }
        }
        const double *ybase = y + P.off * N;

#pragma unroll
        for (int ch = 0; ch < (kMaxN + kCh - 1) / kCh; ++ch) {
            if (ch >= nch) break;
            const int v0 = ch * kCh;
            // 1. stage the footprint of unknowns v0..v0+15: all loads of a
            //    slot are issued before its LDS stores
            {
                double r0[kCh];
#pragma unroll
                for (int vl = 0; vl < kCh; ++vl)
                    r0[vl] = (v0 + vl < N) ? ybase[(long long)(v0 + vl) * C + fo0] : 0.0;
#pragma unroll
                for (int vl = 0; vl < kCh; ++vl) sQ[vl][t] = r0[vl];
            }
            if (has1) {
                double r1[kCh];
#pragma unroll
                for (int vl = 0; vl < kCh; ++vl)
                    r1[vl] = (v0 + vl < N) ? ybase[(long long)(v0 + vl) * C + fo1] : 0.0;
#pragma unroll
                for (int vl = 0; vl < kCh; ++vl) sQ[vl][s1] = r1[vl];
            }
            __syncthreads();
            // 2. gradients and dissipation of the chunk
            for (int e = t; e < kCh * kTC; e += kFdThreads) {
                const int vl = e / kTC, c = e - vl * kTC;
                const int x = c % kT, yy = (c / kT) % kT, z = c / (kT * kT);
                const double *u = sQ[vl];
                const double u0 = u[c];
                double ko = 0.0;
                // x
                {
                    const double m3 = u[foot_slot(x - 3, yy, z)], m2 = u[foot_slot(x - 2, yy, z)],
                                 m1 = u[foot_slot(x - 1, yy, z)], p1 = u[foot_slot(x + 1, yy, z)],
                                 p2 = u[foot_slot(x + 2, yy, z)], p3 = u[foot_slot(x + 3, yy, z)];
                    sG[0][vl][c] = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                // y
                {
                    const double m3 = u[foot_slot(x, yy - 3, z)], m2 = u[foot_slot(x, yy - 2, z)],
                                 m1 = u[foot_slot(x, yy - 1, z)], p1 = u[foot_slot(x, yy + 1, z)],
                                 p2 = u[foot_slot(x, yy + 2, z)], p3 = u[foot_slot(x, yy + 3, z)];
                    sG[1][vl][c] = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                // z
                {
                    const double m3 = u[foot_slot(x, yy, z - 3)], m2 = u[foot_slot(x, yy, z - 2)],
                                 m1 = u[foot_slot(x, yy, z - 1)], p1 = u[foot_slot(x, yy, z + 1)],
                                 p2 = u[foot_slot(x, yy, z + 2)], p3 = u[foot_slot(x, yy, z + 3)];
                    sG[2][vl][c] = ((m2 - p2) + 8.0 * (p1 - m1)) * c4;
                    ko += ((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1) - 20.0 * u0;
                }
                sK[vl][c] = cko * ko;
            }
            __syncthreads();
            // 3. accumulate -B_d G_d over the chunk's K rows on the matrix cores
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int kk = 0; kk < kCh / 4; ++kk) {
                    if (ch * (kCh / 4) + kk >= kMaxN / 4) break;
                    const double aop = a[d][ch * (kCh / 4) + kk];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        accm[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, sG[d][4 * kk + lg][nt * 16 + lj],
                                                                        accm[nt], 0, 0, 0);
                }
            // the chunk whose unknowns are this wave's output rows adds KO6
            if (ch == w) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) accm[nt][i] += sK[lg + 4 * i][nt * 16 + lj];
            }
            __syncthreads();
        }
        // 4. stage update in the output layout, four rows at a time: reads
        //    first, then the arithmetic and the stores
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int c = nt * 16 + lj;
            const int x = c % kT, yy = (c / kT) % kT, z = c / (kT * kT);
            const long long cell = ((long long)(tz + z) * p + (ty + yy)) * p + (tx + x);
            long long gidx[4];
            double q0v[4], accv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * w + lg + 4 * i;
                const bool ok = r < N;
                gidx[i] = P.off * N + (long long)(ok ? r : 0) * C + cell;
                q0v[i] = (ok && (rk == 1 || stage < 3)) ? q0[gidx[i]] : 0.0;
                accv[i] = (ok && rk == 4 && stage > 0) ? acc[gidx[i]] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * w + lg + 4 * i;
                if (r >= N) continue;
                const long long g = gidx[i];
                const double R = accm[nt][i];
                if (rk == 1) {
                    acc[g] = q0v[i] + dt * R;
                } else if (stage == 0) {
                    ynext[g] = q0v[i] + 0.5 * dt * R;
                    acc[g] = q0v[i] + (dt / 6.0) * R;
                } else if (stage == 1) {
                    ynext[g] = q0v[i] + 0.5 * dt * R;
                    acc[g] = accv[i] + (dt / 3.0) * R;
                } else if (stage == 2) {
                    ynext[g] = q0v[i] + dt * R;
                    acc[g] = accv[i] + (dt / 3.0) * R;
                } else {
                    acc[g] = accv[i] + (dt / 6.0) * R;
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
    const int grid = std::max(1, std::min(b->fd_n_items, cus * b->fd_wg_per_cu));
    hipLaunchKernelGGL(fd_stage_kernel, dim3(grid), dim3(kFdThreads), 0, s, static_cast<const double *>(y),
                       static_cast<const double *>(q0), static_cast<double *>(ynext), static_cast<double *>(acc),
                       b->d_patches, reinterpret_cast<const FdItem *>(b->d_fd_items), b->fd_n_items,
                       b->d_fd_B, b->N, stage, rk_stages, dt, sigma, b->fd_xcd_remap);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

}  // namespace pb
