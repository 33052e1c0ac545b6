// Fused separable space-time stencil for gfx950.
//
// One workgroup owns a TH x TW output tile of every frame and streams along
// the time axis. For each input frame it
//   0. (one frame ahead) loads the halo-extended (TH+2RS) x (TW+2RS) input
//      tile with raw buffer loads into registers; out-of-volume offsets fall
//      outside the buffer range and read as 0, which is exactly the zero
//      padding of the operator;
//   1. forms the pass input u with the operation's prologue (u = f * x for
//      the forward step) and stores it to LDS;
//   2. y-pass: each work item filters RY rows of one halo column from LDS and
//      writes them to a second LDS tile;
//   3. x-pass: each thread filters QX consecutive outputs of a row;
//   4. t-pass: scatters those values into 2RT+1 rotating register
//      accumulators, one per output frame the input frame contributes to.
// When the accumulator of frame t - RT is complete it goes through the
// operation's epilogue (z = s * f * acc for the forward step, the store and
// the reduction partials).
//
// Only the small t-scatter/epilogue is specialised per ring position (a
// switch over t mod (2RT+1)), so the code stays compact. Tiles are handed to
// workgroups so that each XCD (workgroups are dealt round-robin over the 8
// XCDs) owns a contiguous band of tile rows: the y-halo rows that adjacent
// tiles share are then read through the same L2.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace stpi {

constexpr int NUM_XCD = 8;
constexpr uint32_t OOB = 0xFFFFFFF0u;  // byte offset that lies outside every buffer

template <class CT>
struct Taps {
    CT gs[2 * 16 + 1];  // spatial taps g(-RS..RS) of the compiled radius, zero beyond r_s
    CT gt[2 * 8 + 1];   // temporal taps g(-RT..RT)
};

// Raw buffer resource over `bytes` bytes at `base`; loads beyond the range
// return 0 and stores beyond it are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <class ST>
struct BufIO;

template <>
struct BufIO<float> {
    static constexpr uint32_t SZ = 4;
    __device__ static __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
    }
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, boff, 0, 0);
    }
    __device__ static __forceinline__ float rounded(float v) { return v; }
    // four consecutive elements (offset need only be element-aligned)
    __device__ static __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, uint32_t boff, float (&v)[4]) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = __uint_as_float(t[e]);
    }
    __device__ static __forceinline__ void store4(__amdgpu_buffer_rsrc_t r, uint32_t boff, const float (&v)[4]) {
        using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
        V4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = __float_as_uint(v[e]);
        __builtin_amdgcn_raw_buffer_store_b128(t, r, boff, 0, 0);
    }
    // store, and return what the store leaves in memory
    __device__ static __forceinline__ float store_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
        store(r, boff, v);
        return v;
    }
    __device__ static __forceinline__ void store4_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff,
                                                          const float (&v)[4], float (&vr)[4]) {
        store4(r, boff, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) vr[e] = v[e];
    }
};

template <>
struct BufIO<bf16> {
    static constexpr uint32_t SZ = 2;
    __device__ static __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
        return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, boff, 0, 0)) << 16);
    }
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_bits(v), r, boff, 0, 0);
    }
    __device__ static __forceinline__ float rounded(float v) {
        return __uint_as_float(((uint32_t)f32_to_bf16_bits(v)) << 16);
    }
    __device__ static __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, uint32_t boff, float (&v)[4]) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0);
        v[0] = __uint_as_float(t[0] << 16);
        v[1] = __uint_as_float(t[0] & 0xffff0000u);
        v[2] = __uint_as_float(t[1] << 16);
        v[3] = __uint_as_float(t[1] & 0xffff0000u);
    }
    __device__ static __forceinline__ void store4(__amdgpu_buffer_rsrc_t r, uint32_t boff, const float (&v)[4]) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        V2 t;
        t[0] = f32x2_to_bf16x2_bits(v[0], v[1]);
        t[1] = f32x2_to_bf16x2_bits(v[2], v[3]);
        __builtin_amdgcn_raw_buffer_store_b64(t, r, boff, 0, 0);
    }
    // store, and return what the store leaves in memory (one rounding)
    __device__ static __forceinline__ float store_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
        const uint16_t b = f32_to_bf16_bits(v);
        __builtin_amdgcn_raw_buffer_store_b16(b, r, boff, 0, 0);
        return __uint_as_float((uint32_t)b << 16);
    }
    __device__ static __forceinline__ void store4_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff,
                                                          const float (&v)[4], float (&vr)[4]) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        V2 t;
        t[0] = f32x2_to_bf16x2_bits(v[0], v[1]);
        t[1] = f32x2_to_bf16x2_bits(v[2], v[3]);
        __builtin_amdgcn_raw_buffer_store_b64(t, r, boff, 0, 0);
        vr[0] = __uint_as_float(t[0] << 16);
        vr[1] = __uint_as_float(t[0] & 0xffff0000u);
        vr[2] = __uint_as_float(t[1] << 16);
        vr[3] = __uint_as_float(t[1] & 0xffff0000u);
    }
};

template <>
struct BufIO<double> {
    static constexpr uint32_t SZ = 8;
    __device__ static __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
    }
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t boff, double v) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, boff, 0, 0);
    }
    __device__ static __forceinline__ double rounded(double v) { return v; }
    // four element loads; an offset that would wrap past 2^32 (boff near the
    // out-of-range marker) stays out of range instead of wrapping into the buffer
    __device__ static __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, uint32_t boff, double (&v)[4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t o = boff + 8u * e;
            v[e] = load(r, o < boff ? OOB : o);
        }
    }
    __device__ static __forceinline__ void store4(__amdgpu_buffer_rsrc_t r, uint32_t boff, const double (&v)[4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t o = boff + 8u * e;
            store(r, o < boff ? OOB : o, v[e]);
        }
    }
    __device__ static __forceinline__ double store_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff, double v) {
        store(r, boff, v);
        return v;
    }
    __device__ static __forceinline__ void store4_rounded(__amdgpu_buffer_rsrc_t r, uint32_t boff,
                                                          const double (&v)[4], double (&vr)[4]) {
        store4(r, boff, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) vr[e] = v[e];
    }
};

// 16-byte vector of LDS elements.
template <class CT>
struct LdsVec {
    static constexpr int N = 16 / (int)sizeof(CT);
    typedef CT type __attribute__((ext_vector_type(16 / sizeof(CT))));
};

// Tile geometry derived from the template parameters.
template <int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
struct Geometry {
    static constexpr int RSA = (RS + 3) & ~3;           // LDS halo of the y-pass output, 16-byte aligned
    static constexpr int NC = TW + 2 * RS;              // columns of the input tile
    static constexpr int NR = TH + 2 * RS;              // rows of the input tile
    static constexpr int NU = NR * NC;                  // input tile elements
    static constexpr int NPF = (NU + NTHR - 1) / NTHR;  // prefetched elements per thread
    static constexpr int LW = TW + 2 * RSA;             // row length of the y-pass output tile
    static constexpr int NRG = TH / RY;                 // row groups per column in the y-pass
    static constexpr int NYI = NC * NRG;                // y-pass work items
    static constexpr int NQ = TW / QX;                  // x groups per row
    static constexpr int NXI = TH * NQ;                 // x-pass work items
    static constexpr int IPT = (NXI + NTHR - 1) / NTHR; // x-pass items per thread
    static constexpr int NTS = 2 * RT + 1;              // temporal accumulator ring
    static constexpr int NUP = (NU + 3) & ~3;           // Y starts 16-byte aligned
    static constexpr int LDS_ELEMS = NUP + TH * LW;
    static_assert(TH % RY == 0, "RY must divide TH");
    static_assert(TW % QX == 0, "QX must divide TW");
    static_assert(NTHR % 64 == 0, "whole wavefronts");
};

// Maps a workgroup to its tile so that each XCD owns a contiguous band of
// tiles (row-major tile order). Returns -1 for workgroups past the last tile.
__device__ __forceinline__ int xcd_tile(int block, int ntiles) {
    const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
    const int t = (block % NUM_XCD) * per + block / NUM_XCD;
    return t < ntiles ? t : -1;
}

// Adds g * v into ring slot SLOT (compile-time index, so the ring stays in
// registers).
template <int SLOT, class CT, int NTS, int IPT, int QX>
__device__ __forceinline__ void ring_fma(CT (&acc)[NTS][IPT][QX], const CT (&v)[IPT][QX], CT g) {
#pragma unroll
    for (int i = 0; i < IPT; ++i)
#pragma unroll
        for (int q = 0; q < QX; ++q) acc[SLOT][i][q] = fma(g, v[i][q], acc[SLOT][i][q]);
}

// Input frame at ring position J feeds output frames tin - dt, dt in [-RT, RT].
template <int J, int DT, int RT, class CT, int IPT, int QX>
__device__ __forceinline__ void ring_scatter(CT (&acc)[2 * RT + 1][IPT][QX], const CT (&v)[IPT][QX],
                                             const Taps<CT> &tp) {
    if constexpr (DT <= RT) {
        constexpr int NTS = 2 * RT + 1;
        ring_fma<((J - DT) % NTS + NTS) % NTS>(acc, v, tp.gt[DT + RT]);
        ring_scatter<J, DT + 1, RT>(acc, v, tp);
    }
}

// t-scatter of one input frame at ring position J, then the epilogue of the
// output frame tout = tin - RT if the block owns it (otherwise only clearing
// its slot: it collected contributions to a frame that does not exist or
// belongs to the previous frame segment).
template <int J, class CT, int RT, int IPT, int QX, class Op, class ORaw>
__device__ __forceinline__ void ring_step(CT (&acc)[2 * RT + 1][IPT][QX], const CT (&v)[IPT][QX],
                                          const Taps<CT> &tp, bool scatter, bool emit, int tout, const Op &op,
                                          const uint32_t (&ooff)[IPT][QX], const ORaw &oraw, double &d1,
                                          double &d2) {
    constexpr int NTS = 2 * RT + 1;
    if (scatter) ring_scatter<J, -RT, RT>(acc, v, tp);
    constexpr int es = ((J - RT) % NTS + NTS) % NTS;
    if (emit) op.emit_frame(tout, acc[es], oraw, ooff, d1, d2);
#pragma unroll
    for (int i = 0; i < IPT; ++i)
#pragma unroll
        for (int q = 0; q < QX; ++q) acc[es][i][q] = CT(0);
}

// y-pass of one work item: RY outputs down a column from RY + 2 RS inputs
// (stride NC in LDS), streamed: each input is added into every output that
// uses it, so only RY accumulators and the value in flight stay live. Each
// output still sums its taps in increasing d.
template <class CT, int RS, int RY, int NC, int LW>
__device__ __forceinline__ void ypass_item(const CT *col, CT *dstp, const Taps<CT> &tp) {
    CT s[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) s[r] = CT(0);
#pragma unroll
    for (int k = 0; k < RY + 2 * RS; ++k) {
        const CT u = col[k * NC];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int d = k - r;
            if (d >= 0 && d <= 2 * RS) s[r] = fma(tp.gs[d], u, s[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) dstp[r * LW] = s[r];
}

// x-pass of one work item: QX outputs along a row from 16-byte LDS reads of
// the window starting RSA - RS before the first tap, streamed the same way.
template <class CT, int RS, int QX, int RSA>
__device__ __forceinline__ void xpass_item(const CT *row, CT (&o)[QX], const Taps<CT> &tp) {
    using V4 = LdsVec<CT>;
    constexpr int NV = (QX + 2 * RSA) / V4::N;
    const typename V4::type *rowp = reinterpret_cast<const typename V4::type *>(__builtin_assume_aligned(row, 16));
#pragma unroll
    for (int q = 0; q < QX; ++q) o[q] = CT(0);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const typename V4::type t4 = rowp[k];
#pragma unroll
        for (int e = 0; e < V4::N; ++e) {
            const int j = k * V4::N + e;  // window index
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const int d = j - q - (RSA - RS);
                if (d >= 0 && d <= 2 * RS) o[q] = fma(tp.gs[d], t4[e], o[q]);
            }
        }
    }
}

// Frame loop unrolled by the ring length: body(J, p) runs for p = 0 .. n-1
// with J = (p + SHIFT) mod NTS as a compile-time constant. Every pass of the
// outer loop walks the ring once, so each ring slot stays in the same
// registers across the back-edge (a runtime ring index makes the compiler
// re-copy the whole ring at every frame).
template <int NTS, int SHIFT, int J, class F>
__device__ __forceinline__ void ring_loop_unroll(int base, int n, F &body) {
    if constexpr (J < NTS) {
        if (base + J < n) body(std::integral_constant<int, ((J + SHIFT) % NTS + NTS) % NTS>{}, base + J);
        ring_loop_unroll<NTS, SHIFT, J + 1>(base, n, body);
    }
}

template <int NTS, int SHIFT, class F>
__device__ __forceinline__ void ring_loop(int n, F &&body) {
    for (int base = 0; base < n; base += NTS) ring_loop_unroll<NTS, SHIFT, 0>(base, n, body);
}

// Frame order of a block that produces output frames [t0, t1) of a clip of T
// frames from input frames [ts, te) = [t0 - RT, t1 + RT) clipped to the clip.
// Walking forward, a range that ends at T completes its last RT output
// frames only after RT more ring steps with no input (the frames past T are
// zero): steps that do nothing but the epilogue. A range that ends at T and
// starts after 0 is walked backward instead: its missing inputs are then the
// ones it never reaches, and its last output frame completes with its last
// input frame. The ring needs no change for that: the temporal taps are even
// in the frame distance (built from its square), so a reversed walk applies
// the same taps. Local step k takes input frame in(k) (while k < nin) and
// completes the ring slot of output frame out(k); the last owned output
// frame completes at step nstep - 1.
template <int RT>
struct FrameWalk {
    int ts, te, nin, fb, dir, nstep;
    __device__ __forceinline__ FrameWalk(int T, int t0, int t1) {
        ts = t0 - RT > 0 ? t0 - RT : 0;
        te = t1 + RT < T ? t1 + RT : T;
        nin = te - ts;
        const bool rev = t1 == T && t0 > 0;
        dir = rev ? -1 : 1;
        fb = rev ? te - 1 : ts;
        nstep = (rev ? te - t0 : t1 - ts) + RT;
    }
    __device__ __forceinline__ int in(int k) const { return fb + dir * k; }
    __device__ __forceinline__ int out(int k) const { return fb + dir * (k - RT); }
};

// Streams one tile through all frames. Op (forward step or adjoint step)
// provides, with ESZ its element size in bytes:
//   template <int NPF> struct Raw                 raw prefetched operands
//   template <int NPF> void fetch(int t, const uint32_t (&boff)[NPF], Raw<NPF> &raw, bool live)
//       issue the loads of frame t at in-frame byte offsets (OOB offsets give 0;
//       an empty range when !live)
//   template <int NPF> CT input(const Raw<NPF> &raw, int k)
//       pass input u of prefetched element k (e.g. f * x)
//   template <int IPT, int QX> struct OutRaw      operands the epilogue reads
//   template <int IPT, int QX> void fetch_out(int t, const uint32_t (&boff)[IPT][QX],
//       OutRaw<IPT, QX> &raw, bool live)  issue the epilogue's loads of output frame t
//       early, in a fixed count of instructions (on an empty range when !live)
//   template <int IPT, int QX> void emit_frame(int t, const CT (&acc)[IPT][QX],
//       const OutRaw<IPT, QX> &raw, const uint32_t (&boff)[IPT][QX], double &d1, double &d2)
//       epilogue of output frame t (OOB offsets are dropped stores, zero sums)
// The block produces output frames [t0, t1) of a clip of T frames; it reads
// input frames [t0 - RT, t1 + RT) clipped to the clip.
template <class CT, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, class Op>
__device__ __forceinline__ void stencil_tile(const Op &op, const Taps<CT> &tp, int T, int t0, int t1, int H, int W,
                                             int x0, int y0, CT *lds, double &d1, double &d2) {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    constexpr int NC = G::NC, NU = G::NU, NPF = G::NPF, LW = G::LW, RSA = G::RSA;
    constexpr int NYI = G::NYI, NQ = G::NQ, NXI = G::NXI, IPT = G::IPT, NTS = G::NTS;
    constexpr uint32_t ESZ = Op::ESZ;
    const int tid = threadIdx.x;
    CT *U = lds;       // [NR][NC] pass input
    CT *Y = lds + G::NUP;  // [TH][LW] y-filtered, 16-byte aligned rows

    // In-frame byte offsets of the input elements this thread stages.
    uint32_t poff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int e = tid + k * NTHR;
        const int r = e / NC, c = e % NC;
        const int gy = y0 - RS + r, gx = x0 - RS + c;
        const bool ok = e < NU && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
        poff[k] = ok ? (uint32_t)(gy * W + gx) * ESZ : OOB;
    }
    // Output voxels owned by this thread in the x-pass and epilogue.
    uint32_t ooff[IPT][QX];
    int orow[IPT], ocol[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = tid + i * NTHR;
        const bool live = item < NXI;
        orow[i] = live ? item / NQ : 0;
        ocol[i] = live ? (item % NQ) * QX : 0;
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int gy = y0 + orow[i], gx = x0 + ocol[i] + q;
            ooff[i][q] = (live && gy < H && gx < W) ? (uint32_t)(gy * W + gx) * ESZ : OOB;
        }
    }

    CT acc[NTS][IPT][QX];
#pragma unroll
    for (int s = 0; s < NTS; ++s)
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) acc[s][i][q] = CT(0);

    const FrameWalk<RT> fw(T, t0, t1);
    typename Op::template Raw<NPF> pf;
    op.template fetch<NPF>(fw.in(0), poff, pf);

    typename Op::template OutRaw<IPT, QX> oraw;
    // local step i takes input frame fw.in(i) (none once past nin) and emits
    // output frame fw.out(i) when the block owns it
    ring_loop<NTS, 0>(fw.nstep, [&](auto ring_pos, int i) __attribute__((always_inline)) {
        constexpr int J = decltype(ring_pos)::value;  // i % NTS
        CT v[IPT][QX];
        const bool live = i < fw.nin;
        const int tout = fw.out(i);
        const bool emit = tout >= t0 && tout < t1;
        if (live) {
            // stage this frame's prefetched input; then the epilogue's operands
            // load while this frame is filtered (after the staging: loads
            // complete in issue order), then the next frame's prefetch
#pragma unroll
            for (int k = 0; k < NPF; ++k) {
                const int e = tid + k * NTHR;
                if (NU % NTHR == 0 || k < NPF - 1 || e < NU) U[e] = op.template input<NPF>(pf, k);
            }
        }
        // both load groups are issued for every frame (on an empty range when
        // not needed), so that the memory-counter waits before each use allow
        // for the younger group instead of draining it
        op.template fetch_out<IPT, QX>(tout, ooff, oraw, emit);
        op.template fetch<NPF>(fw.in(i + 1), poff, pf, i + 1 < fw.nin);
        if (live) {
            __syncthreads();
            // y-pass
            for (int it = tid; it < NYI; it += NTHR) {
                const int c = it % NC;
                const int g = it / NC;
                const CT *col = U + (g * RY) * NC + c;
                CT u[RY + 2 * RS];
#pragma unroll
                for (int k = 0; k < RY + 2 * RS; ++k) u[k] = col[k * NC];
                CT *dstp = Y + (g * RY) * LW + c + (RSA - RS);
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    CT s = CT(0);
#pragma unroll
                    for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], u[r + d], s);
                    dstp[r * LW] = s;
                }
            }
            __syncthreads();
            // x-pass
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                // 16-byte LDS reads: rows of Y and the window start are aligned
                using V4 = LdsVec<CT>;
                constexpr int NV = (QX + 2 * RSA) / V4::N;
                const typename V4::type *rowp = reinterpret_cast<const typename V4::type *>(
                    __builtin_assume_aligned(Y + orow[i] * LW + ocol[i], 16));
                CT w[QX + 2 * RSA];
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const typename V4::type t = rowp[k];
#pragma unroll
                    for (int e = 0; e < V4::N; ++e) w[k * V4::N + e] = t[e];
                }
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    CT s = CT(0);
#pragma unroll
                    for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], w[q + d + RSA - RS], s);
                    v[i][q] = s;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) v[i][q] = CT(0);
        }
        ring_step<J, CT, RT, IPT, QX>(acc, v, tp, live, emit, tout, op, ooff, oraw, d1, d2);
    });
}

// Software-pipelined variant of stencil_tile. Each phase p (one barrier per
// phase) does three frames' worth of different work:
//   stage frame p into U[p % 2] (and issue the loads of frame p + 1),
//   y-pass of frame p - 1 from U[(p - 1) % 2] into Y[(p - 1) % 2],
//   x-pass, t-scatter and epilogue of frame p - 2 from Y[p % 2].
// A buffer written in phase q is read in phase q + 1 and rewritten in phase
// q + 2, after the barrier of phase q + 1, so one barrier per phase suffices.
// y-pass items are dealt to threads from the front, x-pass items from the
// back, so that every wavefront carries a similar share of both.
template <int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
struct PipeGeometry {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    static constexpr int UB = (G::NU + 1 + 3) & ~3;  // one U buffer, one spare slot, 16-byte aligned size
    static constexpr int YB = TH * G::LW;     // one Y buffer
    static constexpr int LDS_ELEMS = 2 * UB + 2 * YB;
    static constexpr int NYT = (G::NYI + NTHR - 1) / NTHR;  // y-pass items per thread
};

template <class CT, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, class Op>
__device__ __forceinline__ void stencil_tile_pipe(const Op &op, const Taps<CT> &tp, int T, int t0, int t1, int H,
                                                  int W, int x0, int y0, CT *lds, double &d1, double &d2) {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    using PG = PipeGeometry<RS, RT, TH, TW, NTHR, RY, QX>;
    constexpr int NC = G::NC, NU = G::NU, NPF = G::NPF, LW = G::LW, RSA = G::RSA;
    constexpr int NYI = G::NYI, NQ = G::NQ, NXI = G::NXI, IPT = G::IPT, NTS = G::NTS, NYT = PG::NYT;
    constexpr uint32_t ESZ = Op::ESZ;
    const int tid = threadIdx.x;
    CT *const U0 = lds;
    CT *const Y0 = lds + 2 * PG::UB;

    uint32_t poff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int e = tid + k * NTHR;
        const int r = e / NC, c = e % NC;
        const int gy = y0 - RS + r, gx = x0 - RS + c;
        const bool ok = e < NU && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
        poff[k] = ok ? (uint32_t)(gy * W + gx) * ESZ : OOB;
    }
    uint32_t ooff[IPT][QX];
    int orow[IPT], ocol[IPT];
    bool olive[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = (NTHR - 1 - tid) + i * NTHR;
        olive[i] = item < NXI;
        orow[i] = olive[i] ? item / NQ : 0;
        ocol[i] = olive[i] ? (item % NQ) * QX : 0;
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int gy = y0 + orow[i], gx = x0 + ocol[i] + q;
            ooff[i][q] = (olive[i] && gy < H && gx < W) ? (uint32_t)(gy * W + gx) * ESZ : OOB;
        }
    }

    CT acc[NTS][IPT][QX];
#pragma unroll
    for (int s = 0; s < NTS; ++s)
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) acc[s][i][q] = CT(0);

    const FrameWalk<RT> fw(T, t0, t1);
    const int nin = fw.nin;  // input frames (local 0 .. nin - 1)
    typename Op::template Raw<NPF> pf;
    op.template fetch<NPF>(fw.in(0), poff, pf);
    typename Op::template OutRaw<IPT, QX> oraw;

    // local frame i is input frame fw.in(i); its output slot holds frame fw.out(i)
    const int nphase = fw.nstep + 2;
    ring_loop<NTS, -2>(nphase, [&](auto ring_pos, int p) __attribute__((always_inline)) {
        constexpr int J = decltype(ring_pos)::value;  // (p - 2) mod NTS
        const int tx = p - 2;  // local frame of the x-pass / ring step
        const int tout = fw.out(tx);
        const bool emit = tx >= 0 && tout >= t0 && tout < t1;
        // stage local frame p; the epilogue's loads are issued after the staged
        // values are consumed (loads complete in issue order)
        if (p < nin) {
            CT *U = U0 + (p & 1) * PG::UB;
#pragma unroll
            for (int k = 0; k < NPF; ++k) {
                const int e = tid + k * NTHR;
                if (NU % NTHR == 0 || k < NPF - 1 || e < NU) U[e] = op.template input<NPF>(pf, k);
            }
        }
        // both load groups in every phase (empty range when not needed): the
        // memory-counter waits then allow for the younger group
        op.template fetch_out<IPT, QX>(tout, ooff, oraw, emit);
        op.template fetch<NPF>(fw.in(p + 1), poff, pf, p + 1 < nin);
        // y-pass of local frame p - 1
        if (p >= 1 && p - 1 < nin) {
            const CT *U = U0 + ((p - 1) & 1) * PG::UB;
            CT *Y = Y0 + ((p - 1) & 1) * PG::YB;
#pragma unroll
            for (int m = 0; m < NYT; ++m) {
                const int it = tid + m * NTHR;
                if (it < NYI) {
                    const int c = it % NC;
                    const int g = it / NC;
                    ypass_item<CT, RS, RY, NC, LW>(U + (g * RY) * NC + c, Y + (g * RY) * LW + c + (RSA - RS), tp);
                }
            }
        }
        // x-pass, t-ring and epilogue of frame p - 2
        if (tx >= 0) {
            CT v[IPT][QX];
            const bool live = tx < nin;
            if (live) {
                const CT *Y = Y0 + (tx & 1) * PG::YB;
#pragma unroll
                for (int i = 0; i < IPT; ++i) xpass_item<CT, RS, QX, RSA>(Y + orow[i] * LW + ocol[i], v[i], tp);
            } else {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
#pragma unroll
                    for (int q = 0; q < QX; ++q) v[i][q] = CT(0);
            }
            ring_step<J, CT, RT, IPT, QX>(acc, v, tp, live, emit, tout, op, ooff, oraw, d1, d2);
        }
        __syncthreads();
    });
}


// Straight-line form of stencil_tile_pipe: the same three-stage schedule, but
// a phase's staging, prefetch, y-pass, x-pass and t-scatter run without
// branches, so the compiler can interleave one pass's LDS reads with another
// pass's FMAs. Out-of-range work is made harmless instead of skipped:
//   - staging past the last input frame writes a U buffer that only a
//     non-live frame reads; the prefetch re-reads the last frame;
//   - lanes past the last y-pass item redo the last item (same values to the
//     same addresses); surplus staging lanes write one spare slot;
//   - the x-pass result of a non-live frame is replaced by zero before the
//     t-scatter.
// Only the epilogue (loads, stores and sums of an owned output frame) is
// conditional.
template <class CT, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, class Op>
__device__ __forceinline__ void stencil_tile_flat(const Op &op, const Taps<CT> &tp, int T, int t0, int t1, int H,
                                                  int W, int x0, int y0, CT *lds, double &d1, double &d2) {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    using PG = PipeGeometry<RS, RT, TH, TW, NTHR, RY, QX>;
    constexpr int NC = G::NC, NU = G::NU, NPF = G::NPF, LW = G::LW, RSA = G::RSA;
    constexpr int NYI = G::NYI, NQ = G::NQ, NXI = G::NXI, IPT = G::IPT, NTS = G::NTS, NYT = PG::NYT;
    constexpr uint32_t ESZ = Op::ESZ;
    const int tid = threadIdx.x;
    CT *const U0 = lds;
    CT *const Y0 = lds + 2 * PG::UB;

    uint32_t poff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int e = tid + k * NTHR;
        const int r = e / NC, c = e % NC;
        const int gy = y0 - RS + r, gx = x0 - RS + c;
        const bool ok = e < NU && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
        poff[k] = ok ? (uint32_t)(gy * W + gx) * ESZ : OOB;
    }
    // only the last staged element can lie past the tile (NPF = ceil(NU / NTHR)):
    // those lanes write the spare slot NU
    const int elast = tid + (NPF - 1) * NTHR < NU ? tid + (NPF - 1) * NTHR : NU;
    // y-pass items of this thread (clamped to the last item)
    int ycol[NYT], yrow0[NYT];
#pragma unroll
    for (int m = 0; m < NYT; ++m) {
        int it = tid + m * NTHR;
        it = it < NYI ? it : NYI - 1;
        ycol[m] = it % NC;
        yrow0[m] = (it / NC) * RY;
    }
    uint32_t ooff[IPT][QX];
    int orow[IPT], ocol[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = (NTHR - 1 - tid) + i * NTHR;
        const bool olive = item < NXI;
        orow[i] = olive ? item / NQ : 0;
        ocol[i] = olive ? (item % NQ) * QX : 0;
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int gy = y0 + orow[i], gx = x0 + ocol[i] + q;
            ooff[i][q] = (olive && gy < H && gx < W) ? (uint32_t)(gy * W + gx) * ESZ : OOB;
        }
    }

    CT acc[NTS][IPT][QX];
#pragma unroll
    for (int s = 0; s < NTS; ++s)
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) acc[s][i][q] = CT(0);

    const FrameWalk<RT> fw(T, t0, t1);
    const int nin = fw.nin;  // input frames (local 0 .. nin - 1)
    typename Op::template Raw<NPF> pf;
    op.template fetch<NPF>(fw.in(0), poff, pf);
    typename Op::template OutRaw<IPT, QX> oraw;

    const int nphase = fw.nstep + 2;
    ring_loop<NTS, -2>(nphase, [&](auto ring_pos, int p) __attribute__((always_inline)) {
        constexpr int J = decltype(ring_pos)::value;  // (p - 2) mod NTS
        const int tx = p - 2;                         // local frame of the x-pass / t-scatter
        const int tout = fw.out(tx);
        const bool emit = tx >= 0 && tout >= t0 && tout < t1;
        const bool xlive = tx >= 0 && tx < nin;
        // stage local frame p, then issue the epilogue's loads (every phase, a
        // valid frame, so the count is fixed) and the prefetch of local frame
        // p + 1 (clamped). Loads complete in issue order: issuing the epilogue's
        // before consuming the prefetch would make the staging wait for them.
        {
            CT *U = U0 + (p & 1) * PG::UB;
#pragma unroll
            for (int k = 0; k < NPF - 1; ++k) U[tid + k * NTHR] = op.template input<NPF>(pf, k);
            U[elast] = op.template input<NPF>(pf, NPF - 1);
            op.template fetch_out_fixed<IPT, QX>(emit ? tout : t0, ooff, oraw);
            const int pn = p + 1 < nin ? p + 1 : nin - 1;
            op.template fetch<NPF>(fw.in(pn), poff, pf);
        }
        // y-pass of local frame p - 1
        {
            const CT *U = U0 + ((p - 1) & 1) * PG::UB;
            CT *Y = Y0 + ((p - 1) & 1) * PG::YB;
#pragma unroll
            for (int m = 0; m < NYT; ++m) {
                const CT *col = U + yrow0[m] * NC + ycol[m];
                CT u[RY + 2 * RS];
#pragma unroll
                for (int k = 0; k < RY + 2 * RS; ++k) u[k] = col[k * NC];
                CT *dstp = Y + yrow0[m] * LW + ycol[m] + (RSA - RS);
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    CT s = CT(0);
#pragma unroll
                    for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], u[r + d], s);
                    dstp[r * LW] = s;
                }
            }
        }
        // x-pass of local frame tx, then its t-scatter
        CT v[IPT][QX];
        {
            const CT *Y = Y0 + (tx & 1) * PG::YB;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                using V4 = LdsVec<CT>;
                constexpr int NV = (QX + 2 * RSA) / V4::N;
                const typename V4::type *rowp = reinterpret_cast<const typename V4::type *>(
                    __builtin_assume_aligned(Y + orow[i] * LW + ocol[i], 16));
                CT w[QX + 2 * RSA];
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const typename V4::type t4 = rowp[k];
#pragma unroll
                    for (int e = 0; e < V4::N; ++e) w[k * V4::N + e] = t4[e];
                }
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    CT s = CT(0);
#pragma unroll
                    for (int d = 0; d <= 2 * RS; ++d) s = fma(tp.gs[d], w[q + d + RSA - RS], s);
                    v[i][q] = xlive ? s : CT(0);
                }
            }
        }
        ring_scatter<J, -RT, RT>(acc, v, tp);
        constexpr int es = ((J - RT) % NTS + NTS) % NTS;
        op.template emit_frame_fixed<IPT, QX>(tout >= t0 ? tout : t0, emit, acc[es], oraw, ooff, d1, d2);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) acc[es][i][q] = CT(0);
        __syncthreads();
    });
}

}  // namespace stpi
