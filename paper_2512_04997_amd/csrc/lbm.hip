// lbm.hip -- fused in-place (AA pattern) D3Q19 collide-and-stream with BGK or
// TRT (Sec. 2.3, Eqs. collAndStream, BGK, trt_populations, TRT, equilibrium),
// partially saturated cells
// (Sec. 2.4, Eqs. psm1, lbePS, bk, btot, forceSF, torqueSF), halfway and
// moving-wall bounce-back and Guo forcing.
//
// Storage: one array of shifted populations g_i = f_i - w_i, [19][N], type S.
//   even step: lane reads g_i at its own cell slot i and writes g*_i to its own
//              slot opp(i);
//   odd step : lane reads g_i from slot opp(i) of cell x - c_i and writes g*_i
//              to slot i of cell x + c_i.
//   A lane reads and writes the same set of addresses in both steps, so the
//   update is race-free in place.  A link through a wall reads / writes the
//   lane's own opposite slot with the moving-wall term (halfway bounce-back).
// Tiles of 64 x 4 x 4 cells: a workgroup of 256 lanes, one x-row per wave
// (coalesced 64-cell rows), four z-planes per lane.  Tiles with registered
// particles run the PSM kernel: particle kinematics staged in LDS, per-cell
// momentum exchange reduced per particle with wave shuffles into LDS (fixed
// order, no floating-point atomics), one partial per (tile, particle).
// The block -> tile mapping keeps consecutive tiles on one XCD.
#include <hip/hip_fp16.h>

#include <utility>

#include "common.h"
#include "lbm.h"
#include "serve.h"

namespace {

// ---------------------------------------------------------------------------
// storage conversions: double, float, bf16 (round to nearest even), fp16
// ---------------------------------------------------------------------------
struct bf16_t {
    unsigned short u;
};

template <typename S, typename C>
struct Conv;
template <>
struct Conv<double, double> {
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <>
struct Conv<float, float> {
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <>
struct Conv<bf16_t, float> {
    __device__ static float ld(bf16_t v) { return __uint_as_float(((unsigned)v.u) << 16); }
    __device__ static bf16_t st(float v) {
        unsigned u = __float_as_uint(v);
        bf16_t r;
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            r.u = (unsigned short)((u >> 16) | 0x40u);
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            r.u = (unsigned short)(u >> 16);
        }
        return r;
    }
};
template <>
struct Conv<_Float16, float> {
    __device__ static float ld(_Float16 v) { return (float)v; }
    __device__ static _Float16 st(float v) { return (_Float16)v; }
};


// streaming stores and loads of populations (each is touched once per pass)
template <typename S>
__device__ inline void st_nt(S* p, S v) { __builtin_nontemporal_store(v, p); }
template <>
__device__ inline void st_nt<bf16_t>(bf16_t* p, bf16_t v) { __builtin_nontemporal_store(v.u, &p->u); }
template <typename S>
__device__ inline S ld_nt(const S* p) { return __builtin_nontemporal_load(p); }
template <>
__device__ inline bf16_t ld_nt<bf16_t>(const bf16_t* p) { bf16_t r; r.u = __builtin_nontemporal_load(&p->u); return r; }
// NT: streaming form (lattices whose population array exceeds the last-level
// cache), else ordinary accesses (smaller lattices stay cached between passes)
template <bool NT, typename S>
__device__ inline void st_pop(S* p, S v) {
    if constexpr (NT) st_nt(p, v);
    else *p = v;
}
template <bool NT, typename S>
__device__ inline S ld_pop(const S* p) {
    if constexpr (NT) return ld_nt(p);
    else return *p;
}
// ---------------------------------------------------------------------------
// collision of one cell in shifted form (g = f - w), compute type C
// ---------------------------------------------------------------------------
template <typename C, bool PSM>
struct Cell {
    C g[19];
    C out[19];
};

template <typename C>
__device__ inline C W(int i) {
    return (C)d3q19_w(i);
}

// moments and equilibrium scalars
template <typename C>
__device__ inline void moments(const C* g, C& drho, C& jx, C& jy, C& jz) {
    drho = (C)0;
    jx = jy = jz = (C)0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        drho += g[i];
        if (d3q19_cx(i) > 0) jx += g[i];
        if (d3q19_cx(i) < 0) jx -= g[i];
        if (d3q19_cy(i) > 0) jy += g[i];
        if (d3q19_cy(i) < 0) jy -= g[i];
        if (d3q19_cz(i) > 0) jz += g[i];
        if (d3q19_cz(i) < 0) jz -= g[i];
    }
}

template <typename C>
__device__ inline C cdot(int i, C x, C y, C z) {
    C r = (C)0;
    if (d3q19_cx(i) > 0) r += x;
    if (d3q19_cx(i) < 0) r -= x;
    if (d3q19_cy(i) > 0) r += y;
    if (d3q19_cy(i) < 0) r -= y;
    if (d3q19_cz(i) > 0) r += z;
    if (d3q19_cz(i) < 0) r -= z;
    return r;
}

// BGK or TRT (+ PSM, + Guo) collision of one cell; MS = maximum solid slots (0:
// fluid only).  Pk[k] = sum_i Omega^s_ik c_i (before the B_k factor).
// The pair (p, pbar) relaxes its even part at omega and its odd part at
// omega_m: post_p = g_p - a neq_p - b neq_pbar with a = (omega + omega_m)/2,
// b = (omega - omega_m)/2 (b = 0 for BGK, which leaves BGK's arithmetic).  The
// Guo source's odd part w 3 c.F takes 1 - omega_m/2, its even part 1 - omega/2.
// Returns the cell density.
template <typename C, int MS>
__device__ inline C collide(const C* g, C* out, C omega, C omega_m, bool forcing, C Fx, C Fy, C Fz, int nk,
                            const C* B, const C (*uk)[3], C (*Pk)[3]) {
    C drho, jx, jy, jz;
    moments(g, drho, jx, jy, jz);
    const C rho = (C)1 + drho;
    const C irho = (C)1 / rho;
    C ux, uy, uz;
    if (forcing) {
        ux = (jx + (C)0.5 * Fx) * irho;
        uy = (jy + (C)0.5 * Fy) * irho;
        uz = (jz + (C)0.5 * Fz) * irho;
    } else {
        ux = jx * irho;
        uy = jy * irho;
        uz = jz * irho;
    }
    const C usq = ux * ux + uy * uy + uz * uz;
    const C E = drho - (C)1.5 * rho * usq;
    C Bt = (C)0;
    C Ek[MS > 0 ? MS : 1];
#pragma unroll
    for (int k = 0; k < MS; ++k) {
        if (k < nk) {
            Bt += B[k];
            const C uk2 = uk[k][0] * uk[k][0] + uk[k][1] * uk[k][1] + uk[k][2] * uk[k][2];
            Ek[k] = drho - (C)1.5 * rho * uk2;
        }
        Pk[k][0] = Pk[k][1] = Pk[k][2] = (C)0;
    }
    Bt = Bt < (C)1 ? Bt : (C)1;
    const C om = MS > 0 ? ((C)1 - Bt) * omega : omega;
    const C fpre = MS > 0 ? ((C)1 - Bt) : (C)1;
    const C wa = (C)0.5 * (omega + omega_m), wb = (C)0.5 * (omega - omega_m);
    const C oa = MS > 0 ? ((C)1 - Bt) * wa : wa;
    const C ob = MS > 0 ? ((C)1 - Bt) * wb : wb;
    const C gk = (C)1 - (C)0.5 * omega;     // even Guo prefactor 1 - (dt/tau+)/2
    const C gkm = (C)1 - (C)0.5 * omega_m;  // odd Guo prefactor 1 - (dt/tau-)/2
    const C uF = ux * Fx + uy * Fy + uz * Fz;
    {
        const C geq0 = W<C>(0) * E;
        C o = g[0] - om * (g[0] - geq0);
        if (forcing) o += fpre * gk * W<C>(0) * ((C)-3 * uF);
#pragma unroll
        for (int k = 0; k < MS; ++k)
            if (k < nk) o += B[k] * (W<C>(0) * (Ek[k] - E));
        out[0] = o;
    }
#pragma unroll
    for (int p = 1; p <= 9; ++p) {
        const int q = p + 9;
        const C w = W<C>(p);
        const C cu = cdot<C>(p, ux, uy, uz);
        const C sym = w * (E + (C)4.5 * rho * cu * cu);
        const C anti = w * (C)3 * rho * cu;
        const C neqp = g[p] - (sym + anti), neqq = g[q] - (sym - anti);
        C op = (g[p] - oa * neqp) - ob * neqq;
        C oq = (g[q] - oa * neqq) - ob * neqp;
        if (forcing) {
            const C cF = cdot<C>(p, Fx, Fy, Fz);
            const C t = gk * ((C)9 * cu * cF - (C)3 * uF);
            const C a3 = gkm * ((C)3 * cF);
            op += fpre * w * (a3 + t);
            oq += fpre * w * (t - a3);
        }
#pragma unroll
        for (int k = 0; k < MS; ++k) {
            if (k < nk) {
                const C cuk = cdot<C>(p, uk[k][0], uk[k][1], uk[k][2]);
                const C symk = w * (Ek[k] + (C)4.5 * rho * cuk * cuk);
                const C antik = w * (C)3 * rho * cuk;
                const C Osp = neqq - (g[p] - (symk + antik));
                const C Osq = neqp - (g[q] - (symk - antik));
                op += B[k] * Osp;
                oq += B[k] * Osq;
                const C d = Osp - Osq;
                if (d3q19_cx(p) > 0) Pk[k][0] += d;
                if (d3q19_cx(p) < 0) Pk[k][0] -= d;
                if (d3q19_cy(p) > 0) Pk[k][1] += d;
                if (d3q19_cy(p) < 0) Pk[k][1] -= d;
                if (d3q19_cz(p) > 0) Pk[k][2] += d;
                if (d3q19_cz(p) < 0) Pk[k][2] -= d;
            }
        }
        out[p] = op;
        out[q] = oq;
    }
    return rho;
}

// Per-axis neighbour offsets (wrapped on periodic axes) and wall flags of a
// lane; a direction's source or destination and the walled face its link
// crosses (lowest face index first) follow with a few selects.
struct AxisNb {
    int om, op;      // element offset of the -1 / +1 neighbour
    bool wl, wh;     // the -1 / +1 neighbour lies beyond a wall
};

__device__ inline AxisNb axis_nb(int c, int n, int periodic, int stride) {
    AxisNb a;
    a.wl = !periodic && c == 0;
    a.wh = !periodic && c == n - 1;
    a.om = c == 0 ? (periodic ? (n - 1) * stride : 0) : -stride;
    a.op = c == n - 1 ? (periodic ? -(n - 1) * stride : 0) : stride;
    return a;
}

template <int DX, int DY, int DZ>
__device__ inline int dir_off(const AxisNb& ax, const AxisNb& ay, const AxisNb& az, int* face) {
    int f = -1;
    if (DX < 0 && ax.wl) f = 0;
    if (DX > 0 && ax.wh) f = 1;
    if (f < 0 && DY < 0 && ay.wl) f = 2;
    if (f < 0 && DY > 0 && ay.wh) f = 3;
    if (f < 0 && DZ < 0 && az.wl) f = 4;
    if (f < 0 && DZ > 0 && az.wh) f = 5;
    *face = f;
    int o = 0;
    if (DX < 0) o += ax.om;
    if (DX > 0) o += ax.op;
    if (DY < 0) o += ay.om;
    if (DY > 0) o += ay.op;
    if (DZ < 0) o += az.om;
    if (DZ > 0) o += az.op;
    return o;
}

template <typename S, typename C, bool ODD, bool NT, int I>
__device__ inline void load_dir(const LbmArgs& A, const S* f, long long N, long long cell, const AxisNb& ax,
                                const AxisNb& ay, const AxisNb& az, C* g) {
    if (!ODD) {
        g[I] = Conv<S, C>::ld(ld_pop<NT>(&f[(long long)I * N + cell]));
    } else {
        int face;
        const int o = dir_off<-d3q19_cx(I), -d3q19_cy(I), -d3q19_cz(I)>(ax, ay, az, &face);
        if (face >= 0) g[I] = Conv<S, C>::ld(f[(long long)I * N + cell]) + (C)A.wall_corr[face * 19 + I];
        else g[I] = Conv<S, C>::ld(f[(long long)d3q19_opp(I) * N + cell + o]);
    }
}

template <typename S, typename C, bool ODD, bool NT, int I>
__device__ inline void store_dir(const LbmArgs& A, S* f, long long N, long long cell, const AxisNb& ax,
                                 const AxisNb& ay, const AxisNb& az, const C* out) {
    if (!ODD) {
        st_pop<NT>(&f[(long long)d3q19_opp(I) * N + cell], Conv<S, C>::st(out[I]));
    } else {
        int face;
        const int o = dir_off<d3q19_cx(I), d3q19_cy(I), d3q19_cz(I)>(ax, ay, az, &face);
        if (face >= 0) st_pop<NT>(&f[(long long)d3q19_opp(I) * N + cell], Conv<S, C>::st(out[I] - (C)A.wall_corr[face * 19 + I]));
        else st_pop<NT>(&f[(long long)I * N + cell + o], Conv<S, C>::st(out[I]));
    }
}

template <typename S, typename C, bool ODD, bool NT, int... Is>
__device__ inline void load_all(const LbmArgs& A, const S* f, long long N, long long cell, const AxisNb& ax,
                                const AxisNb& ay, const AxisNb& az, C* g, std::integer_sequence<int, Is...>) {
    (load_dir<S, C, ODD, NT, Is>(A, f, N, cell, ax, ay, az, g), ...);
}

template <typename S, typename C, bool ODD, bool NT, int... Is>
__device__ inline void store_all(const LbmArgs& A, S* f, long long N, long long cell, const AxisNb& ax,
                                 const AxisNb& ay, const AxisNb& az, const C* out, std::integer_sequence<int, Is...>) {
    (store_dir<S, C, ODD, NT, Is>(A, f, N, cell, ax, ay, az, out), ...);
}

// Rows whose links cross no wall (every row of a periodic domain, and all but
// the edge rows of a walled one): each direction reads and writes its own
// population plane at a 32-bit byte offset from that plane's base, the
// neighbour offsets being the per-axis wrap-aware steps.
template <typename S>
__device__ inline const S* plane_ptr(const S* f, long long N, int i, unsigned off_bytes) {
    return (const S*)((const char*)(f + (long long)i * N) + off_bytes);
}

template <typename S>
__device__ inline S* plane_ptr(S* f, long long N, int i, unsigned off_bytes) {
    return (S*)((char*)(f + (long long)i * N) + off_bytes);
}

template <int DX, int DY, int DZ>
__device__ inline int plain_off(const AxisNb& ax, const AxisNb& ay, const AxisNb& az) {
    int o = 0;
    if (DX < 0) o += ax.om;
    if (DX > 0) o += ax.op;
    if (DY < 0) o += ay.om;
    if (DY > 0) o += ay.op;
    if (DZ < 0) o += az.om;
    if (DZ > 0) o += az.op;
    return o;
}

// XW: x walls are handled per lane: a link leaving through the x face of a lane
// at x = 0 or x = nx - 1 reads / writes the lane's own opposite slot with the
// moving-wall term (faces 0 and 1 are the only ones such a row can cross).
// Waves with no lane at an x wall take XW = false and keep one unconditional
// access per direction.
template <typename S, typename C, bool ODD, bool XW, bool NT, int I>
__device__ inline void load_plain(const LbmArgs& A, const S* f, long long N, unsigned cell, const AxisNb& ax,
                                  const AxisNb& ay, const AxisNb& az, C* g) {
    constexpr unsigned sz = sizeof(S);
    if (!ODD) {
        g[I] = Conv<S, C>::ld(ld_pop<NT>(plane_ptr(f, N, I, cell * sz)));
    } else {
        constexpr int cx = d3q19_cx(I);
        const int o = plain_off<-d3q19_cx(I), -d3q19_cy(I), -d3q19_cz(I)>(ax, ay, az);
        const bool xw = XW && ((cx > 0 && ax.wl) || (cx < 0 && ax.wh));
        if (XW && cx != 0 && xw) {
            const int face = cx > 0 ? 0 : 1;
            g[I] = Conv<S, C>::ld(*plane_ptr(f, N, I, cell * sz)) + (C)A.wall_corr[face * 19 + I];
        } else {
            // links without an x component read whole lines of another row:
            // streamed like the even pass; the x-shifted ones share their
            // boundary lines with the neighbouring waves and stay ordinary
            g[I] = Conv<S, C>::ld(ld_pop<NT && cx == 0>(plane_ptr(f, N, d3q19_opp(I), (unsigned)((int)cell + o) * sz)));
        }
    }
}

template <typename S, typename C, bool ODD, bool XW, bool NT, int I>
__device__ inline void store_plain(const LbmArgs& A, S* f, long long N, unsigned cell, const AxisNb& ax,
                                   const AxisNb& ay, const AxisNb& az, const C* out) {
    constexpr unsigned sz = sizeof(S);
    if (!ODD) {
        st_pop<NT>(plane_ptr(f, N, d3q19_opp(I), cell * sz), Conv<S, C>::st(out[I]));
    } else {
        constexpr int cx = d3q19_cx(I);
        const int o = plain_off<d3q19_cx(I), d3q19_cy(I), d3q19_cz(I)>(ax, ay, az);
        const bool xw = XW && ((cx < 0 && ax.wl) || (cx > 0 && ax.wh));
        if (XW && cx != 0 && xw) {
            const int face = cx < 0 ? 0 : 1;
            st_pop<NT>(plane_ptr(f, N, d3q19_opp(I), cell * sz), Conv<S, C>::st(out[I] - (C)A.wall_corr[face * 19 + I]));
        } else {
            st_pop<NT>(plane_ptr(f, N, I, (unsigned)((int)cell + o) * sz), Conv<S, C>::st(out[I]));
        }
    }
}

template <typename S, typename C, bool ODD, bool XW, bool NT, int... Is>
__device__ inline void load_all_plain(const LbmArgs& A, const S* f, long long N, unsigned cell, const AxisNb& ax,
                                      const AxisNb& ay, const AxisNb& az, C* g, std::integer_sequence<int, Is...>) {
    (load_plain<S, C, ODD, XW, NT, Is>(A, f, N, cell, ax, ay, az, g), ...);
}

template <typename S, typename C, bool ODD, bool XW, bool NT, int... Is>
__device__ inline void store_all_plain(const LbmArgs& A, S* f, long long N, unsigned cell, const AxisNb& ax,
                                       const AxisNb& ay, const AxisNb& az, const C* out,
                                       std::integer_sequence<int, Is...>) {
    (store_plain<S, C, ODD, XW, NT, Is>(A, f, N, cell, ax, ay, az, out), ...);
}

__device__ inline unsigned long long ballot64(bool p) { return __ballot(p); }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Adds, for every distinct particle id among the lanes with has set, the wave
// sum of those lanes' (P, T) into acc[wid][id] (lane 0 writes; a fixed
// butterfly order, no atomics).
__device__ inline void wave_add_by_id(bool has, int my, const double* P, const double* T, double* acc, int wid,
                                      int lane) {
    unsigned long long pending = ballot64(has);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int target = __shfl(my, leader, 64);
        const bool mine = has && my == target;
        double v[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = mine ? P[a] : 0.0;
            v[3 + a] = mine ? T[a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) v[a] = wave_sum(v[a]);
        if (lane == 0)
#pragma unroll
            for (int a = 0; a < 6; ++a) acc[(wid * PSM_PMAX + target) * 6 + a] += v[a];
        pending &= ~ballot64(mine);
    }
}

// MS = 0: tiles without registered particles; MS > 0: tiles with particles
// one tile of one domain (the body shared by the single-domain and the batched kernels)
template <typename S, typename C, bool ODD, int MS, bool NT>
__device__ void lbm_tile(const LbmArgs& A, const long long t, double* kin_s, double* acc) {
    const long long ntiles = A.g.ntiles;
    long long s0 = A.t.tile_start[t], s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    int count = (int)(s1 - s0);
    if (MS > 0) {
        if (count <= 0) return;
        if (count > PSM_PMAX) count = PSM_PMAX;
    } else {
        if (count > 0) return;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    if (MS > 0) {
        for (int u = tid; u < count * 9; u += 256) {
            int k = (int)(A.t.tile_list[s0 + u / 9] >> 32);
            if (k >= A.np) k = 0;
            kin_s[u] = A.kin[9 * k + u % 9];
        }
        for (int u = tid; u < 4 * count * 6; u += 256) {
            const int w = u / (count * 6), r = u % (count * 6);
            acc[w * PSM_PMAX * 6 + r] = 0.0;
        }
        __syncthreads();
    }
    const int tx = (int)(t % A.g.ntx), ty = (int)((t / A.g.ntx) % A.g.nty);
    const int tz = (int)(t / ((long long)A.g.ntx * A.g.nty));
    const int x = tx * PSM_TX + lane, y = ty * PSM_TY + wid;
    const long long N = A.g.N;
    S* f = (S*)A.f;
    const C omega = (C)A.omega, omega_m = (C)A.omega_m;
    const bool forcing = A.forcing != 0;
    const long long plane = ntiles * (long long)PSM_TILE;
    const C* Bslot = (const C*)A.t.slot_B;
    const AxisNb ax = axis_nb(x, A.g.nx, A.g.periodic[0], 1);
    const AxisNb ay = axis_nb(y, A.g.ny, A.g.periodic[1], A.g.nx);
    const bool xy_ok = x < A.g.nx && y < A.g.ny;
    // this wave's row lies next to no y wall (wave-uniform; x walls are handled per lane)
    const bool row_plain = !ay.wl && !ay.wh;
    // some lane of this wave sits at an x wall (only the odd step's plain access differs)
    const bool row_xw = ODD && __ballot(xy_ok && (ax.wl || ax.wh)) != 0ull;

    // Momentum exchange: each lane accumulates its cells' (P, T) over the
    // tile's planes in MS register slots, one per particle id; the wave sums
    // run once per tile (a lane meeting more ids than slots sends the extra
    // term through the wave sum of its plane).
    int aid[MS > 0 ? MS : 1];
    double aP[MS > 0 ? MS : 1][3], aT[MS > 0 ? MS : 1][3];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        aid[s] = -1;
#pragma unroll
        for (int a = 0; a < 3; ++a) aP[s][a] = aT[s][a] = 0.0;
    }

    bool bad = false;  // a density of this lane's cells is not a positive finite number
#pragma unroll 1
    for (int lz = 0; lz < PSM_TZ; ++lz) {
        const int z = tz * PSM_TZ + lz;
        const bool valid = xy_ok && z < A.g.nz;
        int nk = 0;
        C B[MS > 0 ? MS : 1];
        C Pk[MS > 0 ? MS : 1][3];
        int lpk[MS > 0 ? MS : 1];
        if (valid) {
            // the cell's solid slots are loaded with its populations: one round trip
            unsigned lp = 0xffffffffu;
            C Braw[MS > 0 ? MS : 1];
            const long long sl = t * (long long)PSM_TILE + lane + PSM_TX * (wid + PSM_TY * lz);
            if (MS > 0) {
                lp = ld_pop<NT>(&A.t.slot_lp[sl]);
#pragma unroll
                for (int k = 0; k < MS; ++k) Braw[k] = k < A.ms ? ld_pop<NT>(&Bslot[k * plane + sl]) : (C)0;
            }
            const AxisNb az = axis_nb(z, A.g.nz, A.g.periodic[2], A.g.nx * A.g.ny);
            const long long cell = (long long)x + (long long)A.g.nx * ((long long)y + (long long)A.g.ny * z);
            C g[19], out[19];
            const bool plain = row_plain && !az.wl && !az.wh;
            if (plain && !row_xw)
                load_all_plain<S, C, ODD, false, NT>(A, f, N, (unsigned)cell, ax, ay, az, g,
                                                 std::make_integer_sequence<int, 19>{});
            else if (plain)
                load_all_plain<S, C, ODD, true, NT>(A, f, N, (unsigned)cell, ax, ay, az, g,
                                                std::make_integer_sequence<int, 19>{});
            else
                load_all<S, C, ODD, NT>(A, f, N, cell, ax, ay, az, g, std::make_integer_sequence<int, 19>{});
            C Fx = (C)0, Fy = (C)0, Fz = (C)0;
            if (forcing) {
                Fx = (C)A.F[0];
                Fy = (C)A.F[1];
                Fz = (C)A.F[2];
                if (A.kolm_prof) {
                    const int coord = A.kolm_axis == 0 ? x : (A.kolm_axis == 1 ? y : z);
                    const C add = (C)A.kolm_prof[coord];
                    if (A.kolm_dir == 0) Fx += add;
                    else if (A.kolm_dir == 1) Fy += add;
                    else Fz += add;
                }
            }
            C uk[MS > 0 ? MS : 1][3];
            if (MS > 0) {
#pragma unroll
                for (int k = 0; k < MS; ++k) {
                    const unsigned b = (lp >> (8 * k)) & 0xffu;
                    if (k == nk && k < A.ms && b != 0xffu && (int)b < count) {
                        lpk[k] = (int)b;
                        B[k] = Braw[k];
                        const double* kn = kin_s + 9 * b;
                        const double rj[3] = {x + 0.5, y + 0.5, z + 0.5};
                        double d[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            double v = rj[a] - kn[a];
                            if (A.g.periodic[a]) {
                                if (v > 0.5 * A.L[a]) v -= A.L[a];
                                else if (v < -0.5 * A.L[a]) v += A.L[a];
                            }
                            d[a] = v;
                        }
                        // u_k = v_k + w_k x (r_j - r_k)
                        uk[k][0] = (C)(kn[3] + (kn[7] * d[2] - kn[8] * d[1]));
                        uk[k][1] = (C)(kn[4] + (kn[8] * d[0] - kn[6] * d[2]));
                        uk[k][2] = (C)(kn[5] + (kn[6] * d[1] - kn[7] * d[0]));
                        ++nk;
                    }
                }
            }
            const C rho = collide<C, MS>(g, out, omega, omega_m, forcing, Fx, Fy, Fz, nk, B, uk, Pk);
            bad = bad || !(rho > (C)0 && rho < (C)1e30);
            if (plain && !row_xw)
                store_all_plain<S, C, ODD, false, NT>(A, f, N, (unsigned)cell, ax, ay, az, out,
                                                  std::make_integer_sequence<int, 19>{});
            else if (plain)
                store_all_plain<S, C, ODD, true, NT>(A, f, N, (unsigned)cell, ax, ay, az, out,
                                                 std::make_integer_sequence<int, 19>{});
            else
                store_all<S, C, ODD, NT>(A, f, N, cell, ax, ay, az, out, std::make_integer_sequence<int, 19>{});
        }
        if (MS > 0) {
            // per-particle momentum exchange of this plane: wave sums into LDS
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const bool has = k < nk;
                const int my = has ? lpk[k] : -1;
                double P[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
                if (has) {
                    const double Bd = (double)B[k];
#pragma unroll
                    for (int a = 0; a < 3; ++a) P[a] = Bd * (double)Pk[k][a];
                    const double* kn = kin_s + 9 * my;
                    const double rj[3] = {x + 0.5, y + 0.5, tz * PSM_TZ + lz + 0.5};
                    double d[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        double v = rj[a] - kn[a];
                        if (A.g.periodic[a]) {
                            if (v > 0.5 * A.L[a]) v -= A.L[a];
                            else if (v < -0.5 * A.L[a]) v += A.L[a];
                        }
                        d[a] = v;
                    }
                    T[0] = d[1] * P[2] - d[2] * P[1];
                    T[1] = d[2] * P[0] - d[0] * P[2];
                    T[2] = d[0] * P[1] - d[1] * P[0];
                }
                // the lane's slot for this id: a matching one, else the first free one
                bool placed = false;
#pragma unroll
                for (int s = 0; s < MS; ++s) {
                    const bool take = has && !placed && (aid[s] == my || aid[s] < 0);
                    if (take) {
                        aid[s] = my;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            aP[s][a] += P[a];
                            aT[s][a] += T[a];
                        }
                    }
                    placed = placed || take;
                }
                if (__ballot(has && !placed)) wave_add_by_id(has && !placed, my, P, T, acc, wid, lane);
            }
        }
    }
    if (__ballot(bad) && lane == 0 && A.flags) atomicOr(A.flags, (unsigned long long)PSM_FLAG_UNSTABLE);
    if (MS > 0) {
#pragma unroll
        for (int s = 0; s < MS; ++s)
            if (__ballot(aid[s] >= 0)) wave_add_by_id(aid[s] >= 0, aid[s], aP[s], aT[s], acc, wid, lane);
        __syncthreads();
        for (int u = tid; u < count * 6; u += 256) {
            const int p = u / 6, a = u % 6;
            double s = 0.0;
            for (int w = 0; w < 4; ++w) s += acc[(w * PSM_PMAX + p) * 6 + a];
            A.t.partial[(s0 + p) * 6 + a] = s;
        }
    }
}

// the block -> tile mapping keeps consecutive tiles on one XCD
__device__ inline long long xcd_block(long long nblocks) {
    const long long per = (nblocks + 7) / 8;
    return (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// PSM tiles (two slots): four workgroups per CU within 128 registers where it
// measures faster than the natural allocation: the even step of 16-bit and
// float storage (no spill).  The odd step keeps its natural allocation (three
// workgroups; four would spill, slower for float, and for 16-bit storage on
// lattices of many PSM tiles).
template <typename S, bool ODD, int MS>
struct LbmMinBlocks {
    static constexpr int value = (MS == 2 && !ODD && (sizeof(S) == 2 || sizeof(S) == 4)) ? 4 : 1;
};

template <typename S, typename C, bool ODD, int MS, bool NT>
__global__ __launch_bounds__(256, (LbmMinBlocks<S, ODD, MS>::value)) void k_lbm(LbmArgs A) {
    __shared__ double kin_s[MS > 0 ? PSM_PMAX * 9 : 1];
    __shared__ double acc[MS > 0 ? 4 * PSM_PMAX * 6 : 1];
    const long long t = xcd_block(A.g.ntiles);
    if (t >= A.g.ntiles) return;
    lbm_tile<S, C, ODD, MS, NT>(A, t, kin_s, acc);
}

// Both tile kinds in one launch: the branch is uniform over the workgroup (a
// tile's registration count decides it), so a pass is one kernel and the few
// particle-free tiles of a dense suspension share the rounds of the PSM tiles
// instead of a launch of their own.
template <typename S, typename C, bool ODD, int MS, bool NT>
__global__ __launch_bounds__(256, (LbmMinBlocks<S, ODD, MS>::value)) void k_lbm_mixed(LbmArgs A) {
    __shared__ double kin_s[PSM_PMAX * 9];
    __shared__ double acc[4 * PSM_PMAX * 6];
    const long long t = xcd_block(A.g.ntiles);
    if (t >= A.g.ntiles) return;
    const long long s0 = A.t.tile_start[t];
    long long s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    if (s1 > s0) lbm_tile<S, C, ODD, MS, NT>(A, t, kin_s, acc);
    else lbm_tile<S, C, ODD, 0, NT>(A, t, kin_s, acc);
}

// many domains in one launch: map[b] = (job, tile), the job's parity in dyn.odd
template <typename S, typename C, int MS>
__global__ __launch_bounds__(256) void k_lbm_batch(const LbmArgs* __restrict__ jobs, SrvDyn dyn,
                                                   const int2* __restrict__ map, long long nmap) {
    __shared__ double kin_s[MS > 0 ? PSM_PMAX * 9 : 1];
    __shared__ double acc[MS > 0 ? 4 * PSM_PMAX * 6 : 1];
    const long long b = xcd_block(nmap);
    if (b >= nmap) return;
    const int2 m = map[b];
    if (srv_bit(dyn.odd, m.x)) lbm_tile<S, C, true, MS, false>(jobs[m.x], m.y, kin_s, acc);
    else lbm_tile<S, C, false, MS, false>(jobs[m.x], m.y, kin_s, acc);
}

template <typename S, typename C>
hipError_t launch_batch(const LbmArgs* jobs, const SrvDyn& dyn, const int2* map, long long nmap, int ms,
                        hipStream_t s) {
    const unsigned nb = (unsigned)(8 * ((nmap + 7) / 8));
    if (ms == 0) k_lbm_batch<S, C, 0><<<nb, 256, 0, s>>>(jobs, dyn, map, nmap);
    else if (ms <= 2) k_lbm_batch<S, C, 2><<<nb, 256, 0, s>>>(jobs, dyn, map, nmap);
    else k_lbm_batch<S, C, 4><<<nb, 256, 0, s>>>(jobs, dyn, map, nmap);
    return hipGetLastError();
}

template <typename S, typename C, bool NT>
void launch_pass(const LbmArgs& A, int odd, unsigned nblk, hipStream_t s) {
    // without particles no tile holds a registration: the PSM launch is skipped
    // (two slots: one launch for both tile kinds; four slots keep two launches,
    // whose PSM kernel alone already fills the register file)
    const bool psm = A.np > 0;
    if (psm && A.ms <= 2) {
        if (odd) k_lbm_mixed<S, C, true, 2, NT><<<nblk, 256, 0, s>>>(A);
        else k_lbm_mixed<S, C, false, 2, NT><<<nblk, 256, 0, s>>>(A);
    } else if (odd) {
        k_lbm<S, C, true, 0, NT><<<nblk, 256, 0, s>>>(A);
        if (psm) k_lbm<S, C, true, 4, NT><<<nblk, 256, 0, s>>>(A);
    } else {
        k_lbm<S, C, false, 0, NT><<<nblk, 256, 0, s>>>(A);
        if (psm) k_lbm<S, C, false, 4, NT><<<nblk, 256, 0, s>>>(A);
    }
}

// Streaming accesses pay where the population array does not stay in the
// last-level cache (256 MB) from one pass to the next anyway, and where every
// wave's 64-cell row covers whole lines of 4- or 8-byte populations (x extent
// a multiple of 64); on rows that straddle lines, or with 2-byte populations,
// the streamed partial lines measured slower than ordinary accesses.
#define LBM_STREAM_BYTES (192ll << 20)

template <typename S, typename C>
hipError_t launch_step(const LbmArgs& A, int odd, hipStream_t s) {
    const unsigned nblk = (unsigned)(8 * ((A.g.ntiles + 7) / 8));
    const bool stream = 19ll * A.g.N * (long long)sizeof(S) > LBM_STREAM_BYTES && A.g.nx % 64 == 0 && sizeof(S) >= 4;
    if (stream) launch_pass<S, C, true>(A, odd, nblk, s);
    else launch_pass<S, C, false>(A, odd, nblk, s);
    return hipGetLastError();
}

template <typename S, typename C>
__global__ void k_init(S* f, long long N, double rho0) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
#pragma unroll
    for (int i = 0; i < 19; ++i) f[(long long)i * N + c] = Conv<S, C>::st((C)(d3q19_w(i) * (rho0 - 1.0)));
}

template <typename S, typename C>
__global__ void k_to_double(const S* f, long long n, double* out) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) out[c] = (double)Conv<S, C>::ld(f[c]);
}

template <typename S, typename C>
__global__ void k_from_double(S* f, long long n, const double* in) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) f[c] = Conv<S, C>::st((C)in[c]);
}

inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

hipError_t lbm_step(const LbmArgs& A, int precision, int odd, hipStream_t s) {
    switch (precision) {
        case 0: return launch_step<double, double>(A, odd, s);
        case 1: return launch_step<float, float>(A, odd, s);
        case 2: return launch_step<bf16_t, float>(A, odd, s);
        case 3: return launch_step<_Float16, float>(A, odd, s);
    }
    return hipErrorInvalidValue;
}

hipError_t lbm_step_batch(const LbmArgs* jobs, const SrvDyn& dyn, const int2* map, long long nmap, int ms,
                          int precision, hipStream_t s) {
    if (nmap <= 0) return hipSuccess;
    switch (precision) {
        case 0: return launch_batch<double, double>(jobs, dyn, map, nmap, ms, s);
        case 1: return launch_batch<float, float>(jobs, dyn, map, nmap, ms, s);
        case 2: return launch_batch<bf16_t, float>(jobs, dyn, map, nmap, ms, s);
        case 3: return launch_batch<_Float16, float>(jobs, dyn, map, nmap, ms, s);
    }
    return hipErrorInvalidValue;
}

hipError_t lbm_init(void* f, int precision, long long N, double rho0, hipStream_t s) {
    switch (precision) {
        case 0: k_init<double, double><<<nb256(N), 256, 0, s>>>((double*)f, N, rho0); break;
        case 1: k_init<float, float><<<nb256(N), 256, 0, s>>>((float*)f, N, rho0); break;
        case 2: k_init<bf16_t, float><<<nb256(N), 256, 0, s>>>((bf16_t*)f, N, rho0); break;
        case 3: k_init<_Float16, float><<<nb256(N), 256, 0, s>>>((_Float16*)f, N, rho0); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t lbm_to_double(const void* f, int precision, long long n, double* out, hipStream_t s) {
    switch (precision) {
        case 0: k_to_double<double, double><<<nb256(n), 256, 0, s>>>((const double*)f, n, out); break;
        case 1: k_to_double<float, float><<<nb256(n), 256, 0, s>>>((const float*)f, n, out); break;
        case 2: k_to_double<bf16_t, float><<<nb256(n), 256, 0, s>>>((const bf16_t*)f, n, out); break;
        case 3: k_to_double<_Float16, float><<<nb256(n), 256, 0, s>>>((const _Float16*)f, n, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t lbm_from_double(void* f, int precision, long long n, const double* in, hipStream_t s) {
    switch (precision) {
        case 0: k_from_double<double, double><<<nb256(n), 256, 0, s>>>((double*)f, n, in); break;
        case 1: k_from_double<float, float><<<nb256(n), 256, 0, s>>>((float*)f, n, in); break;
        case 2: k_from_double<bf16_t, float><<<nb256(n), 256, 0, s>>>((bf16_t*)f, n, in); break;
        case 3: k_from_double<_Float16, float><<<nb256(n), 256, 0, s>>>((_Float16*)f, n, in); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
