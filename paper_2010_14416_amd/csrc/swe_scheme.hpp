// Device arithmetic of one explicit step shared by the step kernel
// (swe_kernels.hip) and the adjoint kernels (swe_adjoint.hip): the HLLC flux,
// the contributions of one edge, the update of one cell, the decoding of a
// block-edge record, and the per-lane array addressing. Every formula is
// evaluated as written, operation by operation (no contraction: include
// after `#pragma clang fp contract(off)`).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "swe_device.hpp"
#include "swe_mesh.hpp"

namespace swe {

// Element i of an array read or written per lane, addressed as the array's
// base plus a 32-bit byte offset, so that a load takes the base from
// scalar registers and one vector offset register, with no 64-bit address
// arithmetic per lane. Valid while i * sizeof(T) < 2^32: set-up caps a
// mesh (or an ensemble) below 2^29 cells and 2^30 block-edge records, and
// the 8-byte edge arrays are read from their block's first record on.
template <class T>
__device__ __forceinline__ T &at(T *p, int i)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) +
                                  uint32_t(i) * uint32_t(sizeof(T)));
}
template <class T>
__device__ __forceinline__ const T &at(const T *p, int i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                        uint32_t(i) * uint32_t(sizeof(T)));
}

// HLLC flux in the frame of the edge normal (u normal, v tangential).
// A side at or below h_dry is dry: depth and velocities zero. Wave speeds of
// eqs. 19-20 with the star depth of eqs. 21-23 (rarefaction estimate clamped
// at a vacuum), dry-bed speeds of eq. 26, contact speed of eq. 25; the
// tangential momentum flux takes the velocity upwind of the contact.
__device__ __forceinline__ void hllc(double g, double h_dry, double hL,
                                     double uL, double vL, double hR,
                                     double uR, double vR, double &G0,
                                     double &G1, double &G2)
{
    const bool wetL = hL > h_dry, wetR = hR > h_dry;
    if (!wetL) { hL = 0.0; uL = 0.0; vL = 0.0; }
    if (!wetR) { hR = 0.0; uR = 0.0; vR = 0.0; }
    if (!wetL && !wetR) {
        G0 = 0.0; G1 = 0.0; G2 = 0.0;
        return;
    }
    const double aL = sqrt(g * hL), aR = sqrt(g * hR);
    double SL, SR, Ss;
    if (!wetL) {
        SL = uR - 2.0 * aR;
        SR = uR + aR;
        Ss = SL;
    } else if (!wetR) {
        SL = uL - aL;
        SR = uL + 2.0 * aL;
        Ss = SR;
    } else {
        const double hsum = hL + hR;
        const double h0 = 0.5 * hsum - (uR - uL) * hsum / (4.0 * (aL + aR));
        double hs;
        if (h0 <= fmin(hL, hR)) {
            const double b = fmax(0.5 * (aL + aR) + 0.25 * (uL - uR), 0.0);
            hs = b * b / g;
        } else {
            const double gL = sqrt(g * (h0 + hL) / (2.0 * h0 * hL));
            const double gR = sqrt(g * (h0 + hR) / (2.0 * h0 * hR));
            hs = (hL * gL + hR * gR + uL - uR) / (gL + gR);
        }
        const double pL = hs > hL ? sqrt(hs * (hs + hL) / 2.0) / hL : 1.0;
        const double pR = hs > hR ? sqrt(hs * (hs + hR) / 2.0) / hR : 1.0;
        SL = uL - aL * pL;
        SR = uR + aR * pR;
        Ss = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) /
             (hR * (uR - SR) - hL * (uL - SL));
    }
    const double qL = hL * uL, qR = hR * uR;
    if (SL >= 0.0) {
        G0 = qL;
        G1 = qL * uL + 0.5 * g * hL * hL;
        G2 = qL * vL;
    } else if (SR <= 0.0) {
        G0 = qR;
        G1 = qR * uR + 0.5 * g * hR * hR;
        G2 = qR * vR;
    } else {
        const double FL1 = qL * uL + 0.5 * g * hL * hL;
        const double FR1 = qR * uR + 0.5 * g * hR * hR;
        const double rS = 1.0 / (SR - SL);
        G0 = (SR * qL - SL * qR + SR * SL * (hR - hL)) * rS;
        G1 = (SR * FL1 - SL * FR1 + SR * SL * (qR - qL)) * rS;
        G2 = G0 * (Ss >= 0.0 ? vL : vR);
    }
}

struct CellState {
    double h, u, v, z;
};

// Contributions of one edge to its cells' right-hand sides, with F the
// back-rotated flux in the frame of the unit normal n (left to right,
// outward on the boundary) and len the edge length:
// interior edge (left cell L, right cell R): HLLC of the reconstructed
// states (eq. 28; reconstructed depths at or below h_dry count as zero) and
// the bed-slope terms (eq. 30),
//   cl = -len F + len (g/2)(hL**^2 - hL^2)(0, n),
//   cr = +len F - len (g/2)(hR**^2 - hR^2)(0, n);
// boundary edge of cell L: wall, transmissive, inflow of discharge q per
// unit length, or a ghost state of fixed depth / fixed surface elevation
// with the cell's velocity through HLLC, cl = -len F (cr unused).
// One Riemann solve serves every kind.
__device__ __forceinline__ void edge_contrib(double g, double h_dry, bool bnd,
                                             const BcEntry &bc,
                                             const CellState &L,
                                             const CellState &R, double nx,
                                             double ny, double len,
                                             double &cl0, double &cl1,
                                             double &cl2, double &cr0,
                                             double &cr1, double &cr2)
{
    const double unl = L.u * nx + L.v * ny, utl = -L.u * ny + L.v * nx;
    double hl, hr, unr, utr;
    double G0 = 0.0, G1 = 0.0, G2 = 0.0;
    bool solve = true;
    if (!bnd) {
        const double zs = fmax(L.z, R.z);
        hl = L.h - (zs - L.z);
        hr = R.h - (zs - R.z);
        if (hl <= h_dry) hl = 0.0;
        if (hr <= h_dry) hr = 0.0;
        unr = R.u * nx + R.v * ny;
        utr = -R.u * ny + R.v * nx;
    } else {
        hl = L.h;
        unr = unl;
        utr = utl;
        hr = 0.0;
        switch (bc.kind) {
        case 3:   // fixed depth
            hr = bc.value;
            break;
        case 4:   // fixed water-surface elevation
            hr = fmax(bc.value - L.z, 0.0);
            break;
        case 1:   // transmissive
            solve = false;
            G0 = L.h * unl;
            G1 = G0 * unl + 0.5 * g * L.h * L.h;
            G2 = G0 * utl;
            break;
        case 2:   // inflow
            solve = false;
            G0 = -bc.q;
            G1 = (L.h > h_dry ? bc.q * bc.q / L.h : 0.0) +
                 0.5 * g * L.h * L.h;
            G2 = 0.0;
            break;
        default:  // wall
            solve = false;
            G0 = 0.0;
            G1 = 0.5 * g * L.h * L.h;
            G2 = 0.0;
            break;
        }
    }
    if (solve) hllc(g, h_dry, hl, unl, utl, hr, unr, utr, G0, G1, G2);
    const double F1 = G1 * nx - G2 * ny;
    const double F2 = G1 * ny + G2 * nx;
    if (!bnd) {
        const double pl = 0.5 * g * (hl * hl - L.h * L.h);
        const double pr = 0.5 * g * (hr * hr - R.h * R.h);
        cl0 = -len * G0;
        cl1 = len * (pl * nx - F1);
        cl2 = len * (pl * ny - F2);
        cr0 = len * G0;
        cr1 = len * (F1 - pr * nx);
        cr2 = len * (F2 - pr * ny);
    } else {
        cl0 = -len * G0;
        cl1 = -len * F1;
        cl2 = -len * F2;
        cr0 = 0.0;
        cr1 = 0.0;
        cr2 = 0.0;
    }
}

// Update of one cell from the sum R of its three edge contributions:
// dh = dt R_h / A; the semi-implicit Manning solve for dq (eqs. 33-37);
// positivity. `clamp` returns the mass added by the positivity fix.
__device__ __forceinline__ void cell_update(double h_dry, double dt, double A,
                                            double gm2, double h, double hu,
                                            double hv, double R0, double R1,
                                            double R2, double &hn, double &hun,
                                            double &hvn, double &clamp)
{
    const double rA = 1.0 / A;
    const double bh = R0 * rA, bx = R1 * rA, by = R2 * rA;
    const double dh = dt * bh;
    const double qn = sqrt(hu * hu + hv * hv);
    double dqx, dqy;
    if (h > h_dry && qn > 0.0) {
        // semi-implicit Manning: S_f = -c|q|q, c = g m^2 h^(-7/3);
        // (I - dt/2 dS/dq) dq = dt (R_q/A + S_f) + dt/2 (dS/dh) dh
        const double c = gm2 / (h * h * cbrt(h));
        const double sfx = -c * qn * hu, sfy = -c * qn * hv;
        const double rh = 1.0 / h, rq = 1.0 / qn;
        const double jhx = (7.0 / 3.0) * c * qn * hu * rh;
        const double jhy = (7.0 / 3.0) * c * qn * hv * rh;
        const double jxx = -c * (qn + hu * hu * rq);
        const double jxy = -c * hu * hv * rq;
        const double jyy = -c * (qn + hv * hv * rq);
        const double m11 = 1.0 - 0.5 * dt * jxx;
        const double m12 = -0.5 * dt * jxy;
        const double m22 = 1.0 - 0.5 * dt * jyy;
        const double rx = dt * (bx + sfx) + 0.5 * dt * jhx * dh;
        const double ry = dt * (by + sfy) + 0.5 * dt * jhy * dh;
        const double det = m11 * m22 - m12 * m12;
        const double rd = 1.0 / det;
        dqx = (rx * m22 - m12 * ry) * rd;
        dqy = (m11 * ry - m12 * rx) * rd;
    } else {
        dqx = dt * bx;
        dqy = dt * by;
    }
    hn = h + dh;
    hun = hu + dqx;
    hvn = hv + dqy;
    if (hn < 0.0) {
        clamp = -A * hn;
        hn = 0.0;
    }
    if (hn <= h_dry) {
        hun = 0.0;
        hvn = 0.0;
    }
}

// Decoded side of a block edge (see BlockMesh::be_a / be_b).
struct Side {
    int kind;      // 0 cell of this block, 1 cell of another block, 2 boundary
    int local;     // kind 0: local cell index
    int k;         // kind 0: that cell's side along the edge
    int global;    // kind 1: internal cell index; kind 2: boundary slot
};

__device__ __forceinline__ Side decode_side(int32_t v)
{
    Side s;
    const uint32_t u = uint32_t(v);
    if (u & kSideLocal) {
        s.kind = 0;
        s.local = int(u & 0xfffu);
        s.k = int((u >> 12) & 3u);
        s.global = 0;
    } else if (u & kSideBoundary) {
        s.kind = 2;
        s.local = 0;
        s.k = 0;
        s.global = int(u & 0x3fffffffu);
    } else {
        s.kind = 1;
        s.local = 0;
        s.k = 0;
        s.global = v;
    }
    return s;
}

// Time step of this step: CFL * min R/s of U^n, bounded by dt_max, clipped
// to t_end (the last step lands on t_end exactly); dt = 0 once t >= t_end.
struct StepTime {
    double dt, tn;
    long long idx;   // index of this step (from the clock)
    bool unbounded;
};

}  // namespace swe
