// Task numbering of the fluctuation/dissipation sweep: task T in sweep order
// to its cells.  Phase 0 holds one task per cell A (pairs inside A); phase
// 1 + 8 o + pi one task per cell A of coordinate parity pi (pairs between A
// and A + delta_o), in the order tx + hx (ty + hy tz) of A = 2 (tx, ty, tz) +
// parity bits.
#pragma once

#include "sdpd_internal.hpp"

namespace sdpd {

struct TaskCells {
    int64_t A, B;
    int slot;       // 0 = own cell, o + 1 = forward offset o
    int phase;
};

// first task of every phase: 0, ncell, ncell + ncell/8, ...
__device__ __host__ __forceinline__ int64_t phase_base(int64_t ncell, int p)
{
    return p == 0 ? 0 : ncell + (int64_t)(p - 1) * (ncell / 8);
}

// 32-bit index arithmetic throughout: 14 ncell < 2^32 is checked on the host
// (64-bit division is a long software sequence on the GPU)
__device__ __forceinline__ TaskCells task_cells(const DevParams &P, int64_t T64)
{
    TaskCells r;
    const uint32_t T = (uint32_t)T64, ncell = (uint32_t)P.ncell;
    if (T < ncell) {
        r.A = r.B = T;
        r.slot = 0;
        r.phase = 0;
        return r;
    }
    const uint32_t u = T - ncell;
    const uint32_t pq = fast_div(P.div_per, u);
    const uint32_t t = u - pq * P.div_per.d;
    const int p = 1 + (int)pq;
    const int o = (p - 1) / 8, pi = (p - 1) % 8, k = 14 + o;
    const uint32_t txy = fast_div(P.div_hx, t), tx = t - txy * P.div_hx.d;
    const uint32_t tz = fast_div(P.div_hy, txy), ty = txy - tz * P.div_hy.d;
    const int ax = 2 * (int)tx + (pi & 1), ay = 2 * (int)ty + ((pi >> 1) & 1),
              az = 2 * (int)tz + (pi >> 2);
    int bx = ax + k % 3 - 1, by = ay + (k / 3) % 3 - 1, bz = az + k / 9 - 1;
    bx += bx >= P.nc[0] ? -P.nc[0] : (bx < 0 ? P.nc[0] : 0);
    by += by >= P.nc[1] ? -P.nc[1] : (by < 0 ? P.nc[1] : 0);
    bz += bz >= P.nc[2] ? -P.nc[2] : (bz < 0 ? P.nc[2] : 0);
    r.A = (uint32_t)ax + (uint32_t)P.nc[0] * ((uint32_t)ay + (uint32_t)P.nc[1] * (uint32_t)az);
    r.B = (uint32_t)bx + (uint32_t)P.nc[0] * ((uint32_t)by + (uint32_t)P.nc[1] * (uint32_t)bz);
    r.slot = o + 1;
    r.phase = p;
    return r;
}

}  // namespace sdpd
