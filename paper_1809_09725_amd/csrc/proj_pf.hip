// Project-first (PF) FP32 form of the decomposed-time Radon operator and its
// transpose (Sec. 4, eqs. radapr and radadjapr, with the pi-periodicity
// identity and the fold-sum).
//
// Forward  g(i,z,b) = sum_k Phi[i][k] P(a(i), z, b'(i,b), k)
//          P(a,z,b,k) = static projection of f_k at theta0_a in [0,pi)
//          b' = b on even half-turns, Ns-1-b on odd ones (s_{Ns-1-b} = -s_b)
// Adjoint  g~(a,z,b,k) = sum_rot Phi[rot*Ntheta0+a][k] g(rot*Ntheta0+a, z, b')
//          out_k = static back-projection of g~(.,.,.,k) over theta0_a
//
// Kernels
//   k_project      ray-driven projection of a chunk of KC channels for a
//                  group of angle classes of one walk direction; each line
//                  (row or column) of the slice is staged once in LDS and
//                  shared by all rays of the group.
//   k_contract     sum over k with the s-flip; optionally fused with the
//                  h1 prox of Fig. 2 and an FP64 partial of |R f~ - g|^2.
//   k_fold         the fold-sum g -> g~.
// The back-projection of g~ is in backproject.hip.
// Ray positions are computed in FP64 (the rate of FP64 FMA on CDNA4 equals
// that of unpacked FP32), weights and accumulation in FP32.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

constexpr int FT = 512;   // threads of a projection workgroup (8 wave64)
constexpr int G0 = LINE_GUARD;   // zero guard positions at each end of a staged line

// clamp to [0, hi] in one v_med3_i32 (the compiler forms it only for
// constant bounds); hi is uniform and stays in an SGPR
__device__ inline int clamp0_i32(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// clamp to [lo, hi] in one v_med3_i32, both bounds in VGPRs
__device__ inline int clamp_i32(int x, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// Staging of one line (row or column of a slice, KC channels, positions
// 0..N-1 into LDS slots G0..N+G0-1; slots 0..G0-1 and N+G0..N+2G0-1 stay zero)
// through registers: the loads of line l+1 are issued before the taps of line
// l are summed, and written to the other LDS buffer afterwards (or, with one
// buffer, over line l once its taps are done).  PF float4 per thread cover a
// whole line (N * KC <= 4 * PF * NTH).  VEC = 4: float4 loads (K % 4 == 0);
// VEC = 1: scalar loads of the same PF*4 values.  EXACT: the PF float4 of the
// NTH threads are exactly the line's N * KC values and every channel of the
// chunk exists (N * KC == 4 * PF * NTH, K % KC == 0), so the loads need no
// masks; element j of a thread is then at offset off + j * inc of the line
// (32-bit: at most N * N * K < 2^31 floats) and at LDS float dst + j * dinc.
template <int KC, int PF, int VEC, int NTH>
struct LinePrefetch {
    float4 r[PF];
    // EXACT: the offsets of element 0 of this thread (line float, LDS float)
    // and their steps between elements (uniform)
    struct Exact {
        int off, inc, dst, dinc;
    };
    static __device__ inline Exact exact(size_t pstep)
    {
        constexpr int NQ = KC / 4;
        const int pos = threadIdx.x / NQ, kq = threadIdx.x % NQ;
        return {pos * (int)pstep + 4 * kq, (NTH / NQ) * (int)pstep,
                (pos + G0) * line_stride(KC) + 4 * kq, (NTH / NQ) * line_stride(KC)};
    }
    __device__ inline void load(const float *__restrict__ src, size_t pstep, int N, int k0, int K,
                                const Exact &)
    {
        if constexpr (VEC == 4) {
            constexpr int NQ = KC / 4;
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int e = threadIdx.x + NTH * j;
                const int pos = e / NQ, kq = e % NQ;
                r[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (pos < N && k0 + 4 * kq < K) r[j] = *(const float4 *)(src + (size_t)pos * pstep + 4 * kq);
            }
        } else {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = threadIdx.x + NTH * (4 * j + i);
                    const int pos = e / KC, kk = e % KC;
                    v[i] = (pos < N && k0 + kk < K) ? src[(size_t)pos * pstep + kk] : 0.f;
                }
                r[j] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    }
    __device__ inline void store(float *__restrict__ buf, int N, const Exact &) const
    {
        constexpr int stride = line_stride(KC);
        if constexpr (VEC == 4) {
            constexpr int NQ = KC / 4;
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int e = threadIdx.x + NTH * j;
                const int pos = e / NQ, kq = e % NQ;
                if (pos < N) *(float4 *)(buf + (pos + G0) * stride + 4 * kq) = r[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const float v[4] = {r[j].x, r[j].y, r[j].z, r[j].w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = threadIdx.x + NTH * (4 * j + i);
                    const int pos = e / KC, kk = e % KC;
                    if (pos < N) buf[(pos + G0) * stride + kk] = v[i];
                }
            }
        }
    }
};

// What the projection does with its sums P(a,z,b,k): store them (EPI_P), or,
// when one workgroup holds all K channels, contract them with Phi over the
// Npi half-turns with the s-flip (Sec. 4, eq. radapr and the pi-periodicity)
// and store g (EPI_G) or apply the h1 prox of Fig. 2 step 3 (EPI_PROX).
enum { EPI_P = 0, EPI_G = 1, EPI_PROX = 2 };
struct FwdEpi {
    const float *phi;     // [Ntheta][K]
    float *out;           // g (EPI_G) or h1 (EPI_PROX)
    const float *gdata;   // measured sinogram (EPI_PROX)
    double *part;         // per-workgroup FP64 sum of (R f~ - g)^2, or NULL
    float sigma;
    int mode, n0, Npi;
};

// Joseph's ray-driven projection of KC channels of slice z for the rays
// (class, bin) of one group; P(a,z,b,k0..k0+KC) = sum over lines of the
// linear interpolation between the two positions around the ray, times the
// line spacing along the ray 1/c.
// The ray a lane takes: its index pr in the tile, with the bin offset within
// the aligned block of 64 (one wave, one class when BT is a multiple of 64)
// reordered by the class's lane map when there is one.
__device__ inline int fwd_ray(int pr, int a, const unsigned char *__restrict__ lperm)
{
    return lperm && a >= 0 ? (pr & ~63) | (int)lperm[a * 64 + (pr & 63)] : pr;
}

template <int KC, int PPT, int PF, int VEC, bool TL, int NTH, bool EXACT>
__global__ __launch_bounds__(NTH) void k_project(
    const float *__restrict__ f, float *__restrict__ P, const int *__restrict__ gcls,
    const int *__restrict__ gwalk, const unsigned char *__restrict__ lperm,
    const double *__restrict__ ccos, const double *__restrict__ csin, int N, int Nz, int Ns,
    int K, int A, int ngroups, int BT, int nbt, int nkc, int nbuf, unsigned nblocks, FwdEpi E)
{
    constexpr int stride = line_stride(KC);
    extern __shared__ float lines[];   // nbuf buffers x [N + 2 G0 slots][stride], slot = position + G0
    __shared__ double sh[NTH / 64];
    unsigned lid = xcd_remap(blockIdx.x, nblocks);
    const int bt = lid % nbt;
    lid /= nbt;
    const int kc = lid % nkc;
    lid /= nkc;
    const int grp = lid % ngroups;
    const int z = lid / ngroups;
    const int tid = threadIdx.x;
    const int walk = gwalk[grp];
    const int k0 = kc * KC;
    const double hN = 0.5 * (double)(N - 1), hS = 0.5 * (double)(Ns - 1);
    const int bufsz = (N + 2 * G0) * stride;
    if constexpr (EXACT) nbuf = 2;   // planned so (a 512-position line of 16 channels)

    // Ray positions along the lines in 32.32 fixed point: u(l) = u(0) + l s,
    // stepped by an exact integer add per line, so u(l) carries the rounding
    // of u(0) and of l s alone (below 2^-32 (1 + l) positions).  Its integer
    // part gives the left tap (with EXACT, U holds u + G0, so that part is
    // the tap's LDS slot itself), its fraction the interpolation weight.  A
    // ray outside the tile has 1/c = 0; a position before the line or past
    // it is clamped into the zero guard slots.  The unmasked path measured
    // faster with the offset inside U, one 64-bit add per line and the
    // upper bound in an SGPR; the masked path (block sums over 1024
    // positions) measured 3% slower with them and keeps the plain form.
    long long U[PPT], S[PPT];
    float invc[PPT], sfr[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int slot = (tid + NTH * j) / BT;
        const int a = slot < A ? gcls[grp * A + slot] : -1;
        const int b = bt * BT + fwd_ray(tid + NTH * j, a, lperm) % BT;
        double base = -1.0e6, slope = 0.0;
        invc[j] = 0.f;
        if (a >= 0 && b < Ns) {
            const double cs = ccos[a], sn = csin[a], sb = (double)b - hS;
            if (walk == 0) {   // |cos| >= |sin|: the ray crosses every row once
                base = sb / cs + hN;
                slope = -sn / cs;
                invc[j] = (float)(1.0 / fabs(cs));
            } else {           // |sin| > |cos|: every column once
                base = sb / sn + hN;
                slope = -cs / sn;
                invc[j] = (float)(1.0 / fabs(sn));
            }
        }
        const double u0 = fmin(fmax(fma(-hN, slope, base), -1.0e6), 1.0e6);   // line 0
        U[j] = (long long)llrint(u0 * 4294967296.0);
        if constexpr (EXACT) {
            U[j] += (long long)G0 << 32;
            asm volatile("" : "+v"(U[j]));   // keeps the offset inside U (else it is re-added per line)
        }
        S[j] = (long long)llrint(slope * 4294967296.0);
        sfr[j] = invc[j] * 2.3283064365386963e-10f;   // fraction bits -> weight: 2^-32 / c
    }

    // TL (two-level sums, planned for N > 512): the taps of LB consecutive
    // lines go into blk, which is added into acc every LB lines, so that the
    // FP32 rounding of a long ray grows with sqrt(LB) + sqrt(N / LB)
    // additions instead of sqrt(N)
    constexpr int LB = 32;
    float acc[PPT][KC], blk[TL ? PPT : 1][KC];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[j][k] = 0.f;
#pragma unroll
    for (int j = 0; j < (TL ? PPT : 1); ++j)
#pragma unroll
        for (int k = 0; k < KC; ++k) blk[j][k] = 0.f;

    for (int e = tid; e < nbuf * 2 * G0 * stride; e += NTH) {   // zero the guard slots
        const int b = e / (2 * G0 * stride), w = e % (2 * G0 * stride);
        const int row = w / stride;
        lines[b * bufsz + (row < G0 ? row : N + row) * stride + w % stride] = 0.f;
    }

    const size_t lstep = walk == 0 ? (size_t)N * K : (size_t)K;   // next line
    const size_t pstep = walk == 0 ? (size_t)K : (size_t)N * K;   // next position
    const float *src = f + (size_t)z * N * N * K + k0;

    // staging registers: PF float4 per thread, or with EXACT two named float4
    // at the offsets of Stage::exact (an indexed array there is placed in
    // scratch memory by the compiler)
    using Stage = LinePrefetch<KC, PF, VEC, NTH>;
    Stage pf;
    const typename Stage::Exact ex = EXACT ? Stage::exact(pstep) : typename Stage::Exact{0, 0, 0, 0};
    float4 xa, xb;
    auto stage_load = [&]() {
        if constexpr (EXACT) {
            static_assert(PF == 2, "the unmasked staging is planned with 2 float4 per thread");
            xa = *(const float4 *)(src + ex.off);
            xb = *(const float4 *)(src + ex.off + ex.inc);
        } else {
            pf.load(src, pstep, N, k0, K, ex);
        }
    };
    auto stage_store = [&](float *buf) {
        if constexpr (EXACT) {
            *(float4 *)(buf + ex.dst) = xa;
            *(float4 *)(buf + ex.dst + ex.dinc) = xb;
        } else {
            pf.store(buf, N, ex);
        }
    };
    // the taps of every ray on one staged line
    auto line_taps = [&](const float *line) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int q0 = (int)(U[j] >> 32);
            const float fr = (float)(unsigned)U[j];
            U[j] += S[j];
            if constexpr (EXACT)
                asm volatile("" : "+v"(U[j]));   // one 64-bit add per line, not U(0) + l s rebuilt
            const float w1 = fr * sfr[j];
            const float w0 = invc[j] - w1;
            const int slot = EXACT ? clamp0_i32(q0, N + G0) : clamp_i32(q0, -G0, N) + G0;
            const float *t0 = line + __umul24((unsigned)slot, (unsigned)stride);
            // the taps of this ray into s (the ray's sums or its block sums);
            // its FMAs finish before the next ray's tap loads are issued:
            // hoisting the loads of all rays needs 32 VGPRs per ray and spills
            // The left tap's channels are read (and summed) before the right
            // tap's: a wave's consecutive LDS reads then stay on one staged
            // row, which measured 7% faster than alternating the two rows.
            // Each channel still adds w0 x0, then w1 x1.
            auto taps = [&](float (&sr)[KC]) {
#pragma unroll
                for (int k = 0; k < KC; k += 4) {
                    const float4 x0 = *(const float4 *)(t0 + k);
                    sr[k + 0] = fmaf(w0, x0.x, sr[k + 0]);
                    sr[k + 1] = fmaf(w0, x0.y, sr[k + 1]);
                    sr[k + 2] = fmaf(w0, x0.z, sr[k + 2]);
                    sr[k + 3] = fmaf(w0, x0.w, sr[k + 3]);
                }
#pragma unroll
                for (int k = 0; k < KC; k += 4) {
                    const float4 x1 = *(const float4 *)(t0 + stride + k);
                    sr[k + 0] = fmaf(w1, x1.x, sr[k + 0]);
                    sr[k + 1] = fmaf(w1, x1.y, sr[k + 1]);
                    sr[k + 2] = fmaf(w1, x1.z, sr[k + 2]);
                    sr[k + 3] = fmaf(w1, x1.w, sr[k + 3]);
                }
#pragma unroll
                for (int k = 0; k < KC; ++k) asm volatile("" : "+v"(sr[k])::"memory");
            };
            if constexpr (TL) taps(blk[TL ? j : 0]);
            else taps(acc[j]);
        }
    };

    if constexpr (EXACT) {
        // Loads run two lines ahead of the taps (a line's loads have two
        // lines' taps to arrive; one line was too short at one workgroup per
        // CU): two register sets, A and B, alternate over line pairs, and the
        // two LDS buffers alternate as before.  At the taps of line l, line
        // l+1 waits in registers and line l+2 is being loaded.
        static_assert(!TL, "the unmasked staging is planned for N = 512, without block sums");
        constexpr int NL = 512;
        constexpr int bsz = (NL + 2 * G0) * stride;
        // Buffer loads over the slice: the thread's two offsets stay in
        // VGPRs and the line's offset goes in an SGPR, so a load costs no
        // vector address arithmetic.  Every offset is inside the slice
        // (line < NL, element offsets as in LinePrefetch::exact).
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)src, (short)0, (int)(((size_t)N * N * K - k0) * sizeof(float)), 0x00020000);
        const int vo0 = ex.off * (int)sizeof(float), vo1 = (ex.off + ex.inc) * (int)sizeof(float);
        const int lsb = (int)(lstep * sizeof(float));   // bytes per line, < 2^31 / NL
        v4u ra, rb, rc, rd;
        auto ldA = [&](int ln) {
            ra = __builtin_amdgcn_raw_buffer_load_b128(rs, vo0, ln * lsb, 0);
            rb = __builtin_amdgcn_raw_buffer_load_b128(rs, vo1, ln * lsb, 0);
        };
        auto ldB = [&](int ln) {
            rc = __builtin_amdgcn_raw_buffer_load_b128(rs, vo0, ln * lsb, 0);
            rd = __builtin_amdgcn_raw_buffer_load_b128(rs, vo1, ln * lsb, 0);
        };
        auto stA = [&](float *buf) {
            *(v4u *)(buf + ex.dst) = ra;
            *(v4u *)(buf + ex.dst + ex.dinc) = rb;
        };
        auto stB = [&](float *buf) {
            *(v4u *)(buf + ex.dst) = rc;
            *(v4u *)(buf + ex.dst + ex.dinc) = rd;
        };
        ldA(0);
        stA(lines);
        ldB(1);
        __syncthreads();
        // The loads and stores are unconditional (past the end they repeat
        // the last line into a buffer no one reads again): a conditional
        // store would let the compiler sink its loads next to it, and a
        // conditional load would make it wait for every load in flight.
        for (int l = 0; l < NL; l += 2) {
            // line l in buffer 0, line l+1 in B
            ldA(min(l + 2, NL - 1));
            line_taps(lines);
            stB(lines + bsz);
            __syncthreads();
            // line l+1 in buffer 1, line l+2 in A
            ldB(min(l + 3, NL - 1));
            line_taps(lines + bsz);
            stA(lines);
            __syncthreads();
        }
    } else {
    stage_load();
    stage_store(lines);
    __syncthreads();
    for (int l = 0; l < N; ++l) {
        const bool more = l + 1 < N;
        if (more) {
            src += lstep;
            stage_load();
        }
        line_taps(lines + (nbuf == 2 ? (l & 1) * bufsz : 0));
        if constexpr (TL) {
            if ((l + 1) % LB == 0 || !more) {
#pragma unroll
                for (int j = 0; j < PPT; ++j)
#pragma unroll
                    for (int k = 0; k < KC; ++k) {
                        acc[j][k] += blk[TL ? j : 0][k];
                        blk[TL ? j : 0][k] = 0.f;
                    }
            }
        }
        // line l+1 goes to the other buffer while l is read; with one buffer,
        // after every thread's taps of line l
        if (nbuf == 1) __syncthreads();
        if (more) stage_store(lines + (nbuf == 2 ? ((l + 1) & 1) * bufsz : 0));
        __syncthreads();
    }
    }

    double d2 = 0.0;
    const float inv1s = 1.f / (1.f + E.sigma);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int slot = (tid + NTH * j) / BT;
        const int a = slot < A ? gcls[grp * A + slot] : -1;
        const int b = bt * BT + fwd_ray(tid + NTH * j, a, lperm) % BT;
        if (a < 0 || b >= Ns) continue;
        if (E.mode == EPI_P) {
            float *dst = P + (((size_t)a * Nz + z) * Ns + b) * K + k0;
#pragma unroll
            for (int k = 0; k < KC; ++k)
                if (k0 + k < K) dst[k] = acc[j][k];
            continue;
        }
        // every half-turn of class a (K <= KC here); out, gdata and phi do not
        // overlap, so the loads of all half-turns may be issued ahead of the
        // stores
        const float *__restrict__ phi = E.phi;
        const float *__restrict__ gd = E.gdata;
        float *__restrict__ out = E.out;
        // Channels k >= K of the chunk were staged as zeros, so their sums
        // are exactly 0 and a clamped (in-bounds) Phi index leaves v as it
        // is.  The half-turns go in groups of HG whose loads (Phi rows, and
        // for the prox g and h1) are all issued before any of them is used:
        // with one workgroup per CU the epilogue's memory round trips are not
        // hidden by other work, and a branch per channel or a round trip per
        // half-turn cost up to 1 ms per launch.  Lanes past the last
        // half-turn load that half-turn again and store nothing.
        constexpr int HG = KC >= 16 ? 2 : 32 / KC;   // HG * KC <= 32 Phi values in registers
        for (int r0 = 0; r0 < E.Npi; r0 += HG) {
            float ph[HG][KC], gv[HG], hv[HG];
            size_t o[HG];
#pragma unroll
            for (int u = 0; u < HG; ++u) {
                const int r = min(r0 + u, E.Npi - 1);
                const int i = r * E.n0 + a;
                const float *row = phi + (size_t)i * K;
#pragma unroll
                for (int k = 0; k < KC; ++k) ph[u][k] = row[k < K ? k : K - 1];
                o[u] = ((size_t)i * Nz + z) * Ns + ((r & 1) ? Ns - 1 - b : b);
                if (E.mode != EPI_G) {
                    gv[u] = gd[o[u]];
                    hv[u] = out[o[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < HG; ++u) {
                if (r0 + u >= E.Npi) break;
                float v = 0.f;
#pragma unroll
                for (int k = 0; k < KC; ++k) v = fmaf(ph[u][k], acc[j][k], v);
                if (E.mode == EPI_G) {
                    out[o[u]] = v;
                } else {
                    const float d = v - gv[u];
                    d2 += (double)d * (double)d;
                    out[o[u]] = (hv[u] + E.sigma * d) * inv1s;
                }
            }
        }
    }
    if (E.part) {
        const double sum = block_sum(d2, sh);
        if (tid == 0) E.part[blockIdx.x] = sum;
    }
}

// g(i,z,b) = sum_k Phi[i][k] P(a(i), z, b', k); rows (i,z) grid-strided over a
// fixed number of workgroups so the FP64 partials have a fixed order.
__global__ __launch_bounds__(NT) void k_contract(
    const float *__restrict__ P, const float *__restrict__ phi, float *__restrict__ out,
    const float *__restrict__ gdata, int mode, float sigma, double *__restrict__ part, int Nz,
    int Ns, int K, int n0, int Ntheta)
{
    __shared__ double sh[NT / 64];
    const long rows = (long)Ntheta * Nz;
    double d2 = 0.0;
    const float inv1s = 1.f / (1.f + sigma);
    for (long row = blockIdx.x; row < rows; row += gridDim.x) {
        const int i = (int)(row / Nz), z = (int)(row % Nz);
        const int a = i % n0, rot = i / n0;
        const float *ph = phi + (size_t)i * K;
        const float *Pz = P + ((size_t)a * Nz + z) * Ns * K;
        float *o = out + ((size_t)i * Nz + z) * Ns;
        for (int b = threadIdx.x; b < Ns; b += NT) {
            const int bp = (rot & 1) ? Ns - 1 - b : b;
            const float *src = Pz + (size_t)bp * K;
            float v = 0.f;
            if ((K & 3) == 0) {
                for (int k = 0; k < K; k += 4) {
                    const float4 x = *(const float4 *)(src + k);
                    v = fmaf(ph[k], x.x, v);
                    v = fmaf(ph[k + 1], x.y, v);
                    v = fmaf(ph[k + 2], x.z, v);
                    v = fmaf(ph[k + 3], x.w, v);
                }
            } else {
                for (int k = 0; k < K; ++k) v = fmaf(ph[k], src[k], v);
            }
            if (mode == CONTRACT_STORE) {
                o[b] = v;
            } else {   // Fig. 2 step 3: h1 <- (h1 + sigma (R f~ - g)) / (1 + sigma)
                const float d = v - gdata[((size_t)i * Nz + z) * Ns + b];
                d2 += (double)d * (double)d;
                o[b] = (o[b] + sigma * d) * inv1s;
            }
        }
    }
    if (part) {
        const double s = block_sum(d2, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

// g~(a,z,b,k) = sum_rot Phi[rot*n0+a][k] g(rot*n0+a, z, b')  (fold-sum, Sec. 4).
// A workgroup takes one class a and a run of ZB slices: the class's Phi rows
// are staged in LDS once, and each thread owns one bin of one slice: it reads
// the Npi half-turn values of g once each and writes the bin's K channels
// (consecutive threads write consecutive rows of g~).
template <int KB4>   // channels in float4 groups: K <= 4 * KB4
__global__ __launch_bounds__(NT) void k_fold(const float *__restrict__ g,
                                             const float *__restrict__ phi,
                                             float *__restrict__ gt, int Nz, int Ns, int K,
                                             int n0, int Npi, int ZB)
{
    extern __shared__ float sphi[];   // Phi rows of class a: [Npi][4 * KB4], zero padded
    const int nzb = (Nz + ZB - 1) / ZB;
    const int a = blockIdx.x / nzb, z0 = (blockIdx.x % nzb) * ZB;
    constexpr int KP = 4 * KB4;
    for (int e = threadIdx.x; e < Npi * KP; e += NT) {
        const int r = e / KP, k = e % KP;
        sphi[e] = k < K ? phi[(size_t)(r * n0 + a) * K + k] : 0.f;
    }
    __syncthreads();
    const int z1 = min(Nz, z0 + ZB);
    for (int e = threadIdx.x; e < (z1 - z0) * Ns; e += NT) {
        const int z = z0 + e / Ns, b = e % Ns;
        float4 acc[KB4];
#pragma unroll
        for (int q = 0; q < KB4; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int rot = 0; rot < Npi; ++rot) {
            const int i = rot * n0 + a;
            const int bp = (rot & 1) ? Ns - 1 - b : b;
            const float v = g[((size_t)i * Nz + z) * Ns + bp];
            const float4 *ph = (const float4 *)(sphi + rot * KP);
#pragma unroll
            for (int q = 0; q < KB4; ++q) {
                const float4 w = ph[q];
                acc[q].x = fmaf(w.x, v, acc[q].x);
                acc[q].y = fmaf(w.y, v, acc[q].y);
                acc[q].z = fmaf(w.z, v, acc[q].z);
                acc[q].w = fmaf(w.w, v, acc[q].w);
            }
        }
        float *d = gt + (((size_t)a * Nz + z) * Ns + b) * K;
        if ((K & 3) == 0) {
#pragma unroll
            for (int q = 0; q < KB4; ++q)
                if (4 * q < K) *(float4 *)(d + 4 * q) = acc[q];
        } else {
#pragma unroll
            for (int q = 0; q < KB4; ++q) {
                const float c[4] = {acc[q].x, acc[q].y, acc[q].z, acc[q].w};
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (4 * q + t < K) d[4 * q + t] = c[t];
            }
        }
    }
}

template <int KC, int PPT, int PF, int VEC, bool TL, int NTH = FT, bool EXACT = false>
static int launch_project_t(const Plan &p, const float *f, const FwdEpi &E, hipStream_t s,
                            unsigned nb)
{
    const rt_geom &G = p.g;
    const FwdCfg &F = p.fwd;
    auto kern = k_project<KC, PPT, PF, VEC, TL, NTH, EXACT>;
    if (F.lds > 64 * 1024)   // beyond the default dynamic LDS limit: ask for what this plan needs
        RT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)F.lds));
    KTimer kt("k_project", s);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(NTH), F.lds, s, f, p.d_scr, p.d_gcls, p.d_gwalk,
                       F.BT % 64 == 0 ? p.d_lperm : nullptr, p.d_ccos, p.d_csin, G.N, G.Nz, G.Ns, G.K, F.A, F.ngroups, F.BT, F.nbt,
                       F.nkc, F.nbuf, nb, E);
    kt.stop();
    return RT_OK;
}

// two-level sums are planned for N > 512, where 16-channel chunks are not
// used and 8 rays per thread or 8 float4 of prefetch only occur
template <int KC, int PPT, int PF, int VEC>
static int launch_project_l(const Plan &p, const float *f, const FwdEpi &E, hipStream_t s,
                            unsigned nb)
{
    if constexpr (KC == 16) {
        return launch_project_t<KC, PPT, PF, VEC, false>(p, f, E, s, nb);
    } else if constexpr (PPT == 8 || PF == 8) {
        return launch_project_t<KC, PPT, PF, VEC, true>(p, f, E, s, nb);
    } else {
        return p.fwd.tl ? launch_project_t<KC, PPT, PF, VEC, true>(p, f, E, s, nb)
                        : launch_project_t<KC, PPT, PF, VEC, false>(p, f, E, s, nb);
    }
}

template <int KC, int PF, int VEC>
static int launch_project_p(const Plan &p, const float *f, const FwdEpi &E, hipStream_t s,
                            unsigned nb, int ppt)
{
    switch (ppt) {
    case 1: return launch_project_l<KC, 1, PF, VEC>(p, f, E, s, nb);
    case 2: return launch_project_l<KC, 2, PF, VEC>(p, f, E, s, nb);
    case 4: return launch_project_l<KC, 4, PF, VEC>(p, f, E, s, nb);
    default:   // 8 rays per thread: planned only for KC <= 8 with float4 staging
        if constexpr (KC <= 8 && VEC == 4 && PF == 4) {
            return launch_project_l<KC, 8, PF, VEC>(p, f, E, s, nb);
        } else {
            return fail(RT_E_SHAPE, "no projection kernel for 8 rays per thread at KC=%d", KC);
        }
    }
}

template <int KC, int VEC>
static int launch_project_k(const Plan &p, const float *f, const FwdEpi &E, hipStream_t s,
                            unsigned nb, int ppt)
{
    // scalar staging (K % 4 != 0) and 16-channel chunks are planned with 4
    // float4 of prefetch per thread (registers of the two-level ray sums)
    if constexpr (VEC == 1 || KC == 16) {
        return launch_project_p<KC, 4, VEC>(p, f, E, s, nb, ppt);
    } else {
        return p.fwd.pf <= 4 ? launch_project_p<KC, 4, VEC>(p, f, E, s, nb, ppt)
                             : launch_project_p<KC, 8, VEC>(p, f, E, s, nb, ppt);
    }
}

static unsigned row_blocks(long rows) { return (unsigned)std::min<long>(rows, 4096); }

}  // namespace

static unsigned project_blocks(const Plan &p)
{
    const FwdCfg &F = p.fwd;
    return (unsigned)p.g.Nz * F.ngroups * F.nkc * F.nbt;
}

int launch_forward_pf(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                      float *h1, float sigma, double *part, hipStream_t s)
{
    const rt_geom &G = p.g;
    const FwdCfg &F = p.fwd;
    if (G.Nz == 0) return RT_OK;
    const int pairs = F.A * F.BT;
    const int nth = F.nth;
    const int ppt = pairs <= nth ? 1 : pairs <= 2 * nth ? 2 : pairs <= 4 * nth ? 4 : 8;
    const unsigned nb = project_blocks(p);
    const bool fused = F.nkc == 1;   // all K channels in one workgroup: contract in the epilogue
    FwdEpi E{};
    E.phi = p.d_phi;
    E.out = mode == CONTRACT_STORE ? g : h1;
    E.gdata = gdata;
    E.part = fused ? part : nullptr;
    E.sigma = sigma;
    E.mode = !fused ? EPI_P : (mode == CONTRACT_STORE ? EPI_G : EPI_PROX);
    E.n0 = p.n0;
    E.Npi = G.Npi;
    int rc;
    if (nth == 2 * FT) {
        // 16 waves of 2 rays: planned only for 16-channel float4 staging of
        // lines of at most 512 positions (2 float4 of prefetch per thread)
        if (F.vec != 4 || F.KC != 16 || ppt != 2 || F.tl || G.N * 16 > 4 * 2 * 2 * FT)
            return fail(RT_E_SHAPE, "no 1024-thread projection kernel for this plan");
        // the 2 float4 of the 1024 threads are exactly a line of 512 positions
        // when N = 512 and every chunk holds 16 channels: unmasked staging
        if (G.N == 512 && G.K % 16 == 0)
            rc = launch_project_t<16, 2, 2, 4, false, 2 * FT, true>(p, f, E, s, nb);
        else
            rc = launch_project_t<16, 2, 2, 4, false, 2 * FT>(p, f, E, s, nb);
    } else if (F.vec == 4) {
        switch (F.KC) {
        case 4: rc = launch_project_k<4, 4>(p, f, E, s, nb, ppt); break;
        case 8: rc = launch_project_k<8, 4>(p, f, E, s, nb, ppt); break;
        default: rc = launch_project_k<16, 4>(p, f, E, s, nb, ppt); break;
        }
    } else {
        switch (F.KC) {   // the plan keeps KC <= 8 with scalar staging
        case 4: rc = launch_project_k<4, 1>(p, f, E, s, nb, ppt); break;
        case 8: rc = launch_project_k<8, 1>(p, f, E, s, nb, ppt); break;
        default: return fail(RT_E_SHAPE, "no scalar-staging projection for KC=%d", F.KC);
        }
    }
    if (rc) return rc;
    RT_HIP(hipGetLastError());
    if (fused) return RT_OK;
    const unsigned nbc = row_blocks((long)G.Ntheta * G.Nz);
    KTimer kt("k_contract", s);
    hipLaunchKernelGGL(k_contract, dim3(nbc), dim3(NT), 0, s, p.d_scr, p.d_phi, E.out, gdata,
                       mode, sigma, part, G.Nz, G.Ns, G.K, p.n0, G.Ntheta);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int forward_partials(const Plan &p)
{
    if (p.form == RT_FORM_SF) return (int)sf_partials(p);
    return p.fwd.nkc == 1 ? (int)project_blocks(p) : (int)row_blocks((long)p.g.Ntheta * p.g.Nz);
}

int launch_forward(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                   float *h1, float sigma, double *part, hipStream_t s)
{
    if (p.form == RT_FORM_SF) return launch_forward_sf(p, f, g, mode, gdata, h1, sigma, part, s);
    return launch_forward_pf(p, f, g, mode, gdata, h1, sigma, part, s);
}

int launch_adjoint(const Plan &p, const float *g, float *out, hipStream_t s)
{
    if (p.form == RT_FORM_SF) {
        int rc = launch_fold_mfma(p, g, s);
        return rc ? rc : launch_backproject(p, out, s);
    }
    return launch_adjoint_pf(p, g, out, s);
}

int launch_adjoint_pf(const Plan &p, const float *g, float *out, hipStream_t s)
{
    const rt_geom &G = p.g;
    if (G.Nz == 0) return RT_OK;
    // a workgroup per class and run of ZB slices (about 4 bins per thread)
    const int ZB = std::max(1, std::min(G.Nz, 4 * NT / std::max(1, G.Ns)));
    const unsigned nbf = (unsigned)p.n0 * ((G.Nz + ZB - 1) / ZB);
    const int kb4 = (G.K + 3) / 4;
    const size_t lds = (size_t)G.Npi * 4 * (kb4 <= 2 ? 2 : kb4 <= 4 ? 4 : kb4 <= 8 ? 8 : 16) * sizeof(float);
    KTimer kt("k_fold", s);
#define RT_FOLD(B) hipLaunchKernelGGL(k_fold<B>, dim3(nbf), dim3(NT), lds, s, g, p.d_phi, p.d_scr, \
                                      G.Nz, G.Ns, G.K, p.n0, G.Npi, ZB)
    if (kb4 <= 2) RT_FOLD(2);
    else if (kb4 <= 4) RT_FOLD(4);
    else if (kb4 <= 8) RT_FOLD(8);
    else RT_FOLD(16);
#undef RT_FOLD
    kt.stop();
    RT_HIP(hipGetLastError());
    return launch_backproject(p, out, s);
}

}  // namespace rt
