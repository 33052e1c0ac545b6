// Fused separable space-time stencil for gfx950.
//
// One workgroup owns a TH x TW output tile of every frame and streams along
// the time axis. For each input frame it
//   1. y-pass: each work item owns one halo-extended column strip, loads the
//      RY + 2RS input values it needs straight from global memory (coalesced
//      across the wavefront along x), forms the pass input u with the
//      operation's prologue (e.g. u = f * x), and writes the RY vertically
//      filtered values to LDS;
//   2. x-pass: each thread owns IPT groups of QX consecutive outputs of one
//      row and filters horizontally from a 16-byte aligned LDS window;
//   3. t-pass: scatters the 2D-filtered values into 2RT+1 rotating register
//      accumulators (one per output frame the input frame contributes to).
// When the accumulator of frame t - RT is complete it goes through the
// operation's epilogue (e.g. z = s * f * acc, store, reduction partials).
//
// The y-halo is consumed by the y-pass itself, so the only redundant work is
// the y-pass over the 2RS halo columns of the x-pass. Zero padding is exact:
// out-of-volume inputs contribute 0 and the time stream runs RT frames past
// the end. Every frame is updated (no edge frames are left out).
#pragma once

#include "common.hpp"

namespace stpi {

constexpr int QX = 4;  // consecutive x outputs per thread item (one 16-byte LDS chunk)

template <class CT>
struct Taps {
    CT gs[2 * 16 + 1];  // spatial taps g(-r_s..r_s), zero beyond the radius
    CT gt[2 * 8 + 1];   // temporal taps g(-r_t..r_t)
};

// Tile geometry derived from the template parameters.
template <int RS, int RT, int TH, int TW, int NTHR, int RY>
struct Geometry {
    static constexpr int RSA = (RS + 3) & ~3;      // LDS halo, rounded for 16-byte alignment
    static constexpr int NC = TW + 2 * RS;         // columns the y-pass produces
    static constexpr int LW = TW + 2 * RSA;        // LDS row length
    static constexpr int NRG = TH / RY;            // row groups per column in the y-pass
    static constexpr int NYI = NC * NRG;           // y-pass work items
    static constexpr int NQ = TW / QX;             // x groups per row
    static constexpr int NXI = TH * NQ;            // x-pass work items
    static constexpr int IPT = NXI / NTHR;         // x-pass items per thread
    static constexpr int NTS = 2 * RT + 1;         // temporal accumulator ring
    static_assert(TH % RY == 0, "RY must divide TH");
    static_assert(TW % QX == 0, "QX must divide TW");
    static_assert(NXI % NTHR == 0, "x-pass items must be a multiple of the workgroup size");
    static_assert(NTHR % 64 == 0, "whole wavefronts");
};

// Streams one tile through all frames. Op provides
//   CT   load_u(size_t idx)                       pass input at a voxel
//   void emit(size_t idx, CT acc, double &p1, double &p2)
//                                                 epilogue at an output voxel,
//                                                 adding to the per-thread sums
// d1, d2 (double).
template <class CT, int RS, int RT, int TH, int TW, int NTHR, int RY, class Op>
__device__ __forceinline__ void stencil_tile(const Op &op, const Taps<CT> &tp, int T, int H, int W,
                                             int x0, int y0, CT *lds, double &d1, double &d2) {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY>;
    constexpr int RSA = G::RSA, NC = G::NC, LW = G::LW, NYI = G::NYI, NQ = G::NQ;
    constexpr int IPT = G::IPT, NTS = G::NTS;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)H * W;

    CT acc[NTS][IPT][QX];
#pragma unroll
    for (int s = 0; s < NTS; ++s)
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) acc[s][i][q] = CT(0);

    // Output positions owned by this thread in the x-pass / epilogue.
    int orow[IPT], ocol[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = tid + i * NTHR;
        orow[i] = item / NQ;
        ocol[i] = (item % NQ) * QX;
    }

    const int tend = T + RT;
    for (int tb = 0; tb < tend; tb += NTS) {
#pragma unroll
        for (int j = 0; j < NTS; ++j) {
            const int tin = tb + j;
            if (tin >= tend) break;
            if (tin < T) {
                CT *buf = lds + (tin & 1) * (TH * LW);
                const size_t foff = (size_t)tin * plane;
                // ---- y-pass: global -> registers -> LDS
                for (int it = tid; it < NYI; it += NTHR) {
                    const int c = it % NC;
                    const int g = it / NC;
                    const int gx = x0 - RS + c;
                    const bool colok = (unsigned)gx < (unsigned)W;
                    const int ybase = y0 + g * RY - RS;
                    CT u[RY + 2 * RS];
#pragma unroll
                    for (int k = 0; k < RY + 2 * RS; ++k) {
                        const int gy = ybase + k;
                        CT v = CT(0);
                        if (colok && (unsigned)gy < (unsigned)H) v = op.load_u(foff + (size_t)gy * W + gx);
                        u[k] = v;
                    }
                    CT *dstp = buf + (g * RY) * LW + c + (RSA - RS);
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        CT s = CT(0);
#pragma unroll
                        for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], u[r + d], s);
                        dstp[r * LW] = s;
                    }
                }
                __syncthreads();
                // ---- x-pass: LDS -> registers, then t-scatter into the ring
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const CT *rowp = buf + orow[i] * LW + ocol[i];
                    CT w[QX + 2 * RSA];
#pragma unroll
                    for (int k = 0; k < QX + 2 * RSA; ++k) w[k] = rowp[k];
#pragma unroll
                    for (int q = 0; q < QX; ++q) {
                        CT s = CT(0);
#pragma unroll
                        for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], w[q + d + RSA - RS], s);
                        // input frame tin feeds output frames tin - dt, dt in [-RT, RT]
#pragma unroll
                        for (int dt = -RT; dt <= RT; ++dt) {
                            const int slot = ((j - dt) % NTS + NTS) % NTS;
                            acc[slot][i][q] = fma(tp.gt[dt + RT], s, acc[slot][i][q]);
                        }
                    }
                }
            }
            // ---- epilogue for the completed output frame tin - RT. For tin < RT
            // that frame lies before the clip: its slot only collected
            // contributions to a non-existent output and is cleared for reuse.
            if (tin < RT) {
                const int slot = ((j - RT) % NTS + NTS) % NTS;
#pragma unroll
                for (int i = 0; i < IPT; ++i)
#pragma unroll
                    for (int q = 0; q < QX; ++q) acc[slot][i][q] = CT(0);
            } else {
                const int tout = tin - RT;
                const int slot = ((j - RT) % NTS + NTS) % NTS;
                const size_t foff = (size_t)tout * plane;
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const int gy = y0 + orow[i];
#pragma unroll
                    for (int q = 0; q < QX; ++q) {
                        const int gx = x0 + ocol[i] + q;
                        if (gy < H && gx < W) op.emit(foff + (size_t)gy * W + gx, acc[slot][i][q], d1, d2);
                        acc[slot][i][q] = CT(0);
                    }
                }
            }
        }
    }
}

}  // namespace stpi
