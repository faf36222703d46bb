// grpic_qed.hpp -- photon emission and pair conversion of the monopole
// workload (Sec. 4; eq. optical-depth), applied to a particle's end state
// after its push, and the wave-aggregated append of the particles it makes.
//
// Readings of the paper's verbal description:
//   - an e+- whose FIDO Lorentz factor Gamma = sqrt(1 + u^2), u^2 =
//     gamma^ij u_i u_j at its end point, exceeds gamma_thr emits one photon
//     of FIDO energy eps_ph along its momentum; its momentum magnitude drops
//     by eps_ph;
//   - a photon (FIDO energy eps = |u|, at least twice the rest energy)
//     converts with probability P = 1 - exp(-tau dt) into an e- and an e+
//     of energy eps/2 each along its direction, and is removed;
//   - created particles sit at the parent's end point with its weight.
#pragma once

#include "grpic_device.hpp"

namespace grpic {

// Particles a tiled workgroup (one slice) stages in the workspace; those
// beyond go straight to the arrays with one global atomic each.
constexpr int kQedStage = 16;

// The workspace of the staged path (SoA, kQedStage entries per slice).
struct QedStage {
    unsigned long long* count;                // [slices + 1]: staged per slice, then scanned in place
    unsigned long long* blocksums;            // the scan's
    unsigned* ev;                             // [2][slices]: emitted, converted per slice
    int32_t* cell;
    double *xr, *xth, *ur, *uth, *uph, *w;
    uint8_t* sp;
    uint64_t* tag;
};

struct QedArgs {
    double gamma_thr, eps_ph, P;              // P = 1 - exp(-tau dt), formed on the host
    uint64_t seed, step;
    int electron_sp, positron_sp, photon_sp;
    uint64_t* tag;
    int64_t* n_used;                          // [0] elements in use (fixed during the push), [1] appended
    int64_t cap;                              // capacity of the particle arrays
    const int64_t* tail_start;                // tiled: the sort's live count (NULL: 0)
    unsigned long long* qcounters;            // optional: emitted, converted, dropped
    int staged;                               // tiled slices stage their created particles in st
    int64_t slices;                           // slice table entries (staged path)
    QedStage st;
};

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
//   (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
// with the key bumped by the Weyl increments after each round.
struct Philox4 {
    uint64_t v[4];
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                 uint64_t k1) {
    constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
    constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull, kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t h0 = __umul64hi(kMul0, c0), l0 = kMul0 * c0;
        const uint64_t h1 = __umul64hi(kMul1, c2), l1 = kMul1 * c2;
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Up to two particles made by one parent in one step: they share the
// parent's end point and weight and one momentum vector.
struct Created {
    int n;                                    // 0, 1 (a photon) or 2 (e-, e+)
    int cell;
    double xr, xth, w, u[3];
    int sp[2];
    uint64_t tag[2];
};

struct QedEvents {
    int emitted, converted;
};

// Emission or conversion for a particle of species s, tag `tag`, weight w
// whose step left it alive at cell / offsets / momenta `out` (kind 2, x =
// xr, xth, u_r, u_th, u_ph).  Updates out (an emitter's recoil; a
// converted photon becomes kind 1, removed) and fills cr.
template <class Out>
__device__ __forceinline__ void qed_after_step(const StepArgs& A, const QedArgs& Q, int s, uint64_t tag, double w,
                                               Out& out, Created& cr, QedEvents& qe) {
    cr.n = 0;
    if (out.kind != 2) return;
    const bool lepton = s == Q.electron_sp || s == Q.positron_sp;
    const bool photon = s == Q.photon_sp;
    if (!lepton && !photon) return;
    // metric at the stored end point (cell corner + offsets), library functions
    const int i1 = div_by(out.cell, A.nth, A.inv_nth), j1 = out.cell - i1 * A.nth;
    const double xi = (double)i1 + out.x[0], eta = (double)j1 + out.x[1];
    const double r = exp(A.lnr0 + xi * A.dlnr);
    double sn, cs;
    sincos(eta * A.dth, &sn, &cs);
    Metric<double> k;
    ks_metric<double>(A.a, A.M, r, sn, cs, k);
    double u[3] = {out.x[2], out.x[3], out.x[4]};
    const double uu = k.h_rr * u[0] * u[0] + 2.0 * k.h_rp * u[0] * u[2] + k.h_tt * u[1] * u[1] + k.h_pp * u[2] * u[2];
    const double umag = sqrt(uu);
    const bool emits = lepton && sqrt(1.0 + uu) > Q.gamma_thr;
    if (!emits && !photon) return;
    const Philox4 rn = philox4x64_10(tag, Q.step, 0ull, 0ull, Q.seed, 0ull);
    cr.cell = out.cell;
    cr.xr = out.x[0];
    cr.xth = out.x[1];
    cr.w = w;
    if (emits) {
        const double fph = Q.eps_ph / umag, fkeep = (umag - Q.eps_ph) / umag;
        for (int c = 0; c < 3; ++c) {
            cr.u[c] = u[c] * fph;
            out.x[2 + c] = u[c] * fkeep;
        }
        cr.n = 1;
        cr.sp[0] = Q.photon_sp;
        cr.tag[0] = rn.v[1];
        qe.emitted = 1;
        return;
    }
    // a photon: U in [0, 1) from the top 53 bits of the first word
    const double U = (double)(rn.v[0] >> 11) * 0x1.0p-53;
    if (!(U < Q.P && umag >= 2.0)) return;
    const double f = sqrt(0.25 * uu - 1.0) / umag;          // |u| of each lepton over the photon's
    for (int c = 0; c < 3; ++c) cr.u[c] = u[c] * f;
    cr.n = 2;
    cr.sp[0] = Q.electron_sp;
    cr.tag[0] = rn.v[1];
    cr.sp[1] = Q.positron_sp;
    cr.tag[1] = rn.v[2];
    out.kind = 1;
    qe.converted = 1;
}

// Appends the wave's created particles: one atomic per wave reserves their
// range after the elements in use (n0 = n_used[0] at the start of the step);
// those beyond the capacity are dropped.  Every lane of the wave calls it.
template <class T>
__device__ __forceinline__ void qed_append(const StepArgs& A, const QedArgs& Q, int64_t n0, const Created& cr,
                                           const QedEvents& qe) {
    const unsigned long long b1 = __ballot(cr.n & 1), b2 = __ballot(cr.n >> 1);
    const unsigned long long be = __ballot(qe.emitted), bc = __ballot(qe.converted);
    const int lane = threadIdx.x & 63;
    if ((b1 | b2) != 0) {                                     // wave-uniform
        const unsigned long long below = (1ull << lane) - 1ull;
        const int total = __popcll(b1) + 2 * __popcll(b2);
        const int before = __popcll(b1 & below) + 2 * __popcll(b2 & below);
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(Q.n_used + 1), (unsigned long long)total);
        base = __shfl(base, 0);
        int dropped = 0;
        auto put = [&](int64_t q, int sp, uint64_t tag) {
            if (q >= Q.cap) {
                ++dropped;
                return;
            }
            A.cell[q] = cr.cell;
            static_cast<T*>(A.xr)[q] = T(cr.xr);
            static_cast<T*>(A.xth)[q] = T(cr.xth);
            static_cast<T*>(A.ur)[q] = T(cr.u[0]);
            static_cast<T*>(A.uth)[q] = T(cr.u[1]);
            static_cast<T*>(A.uph)[q] = T(cr.u[2]);
            static_cast<T*>(A.w)[q] = T(cr.w);
            const_cast<uint8_t*>(A.sp)[q] = (uint8_t)sp;
            Q.tag[q] = tag;
            if (A.phi) static_cast<T*>(A.phi)[q] = T(0);
        };
        const int64_t q0 = n0 + (int64_t)base + before;
        if (cr.n >= 1) put(q0, cr.sp[0], cr.tag[0]);
        if (cr.n == 2) put(q0 + 1, cr.sp[1], cr.tag[1]);
        if (Q.qcounters) {
            const unsigned long long bd = __ballot(dropped > 0), bd2 = __ballot(dropped > 1);
            if (lane == 0 && (bd | bd2)) atomicAdd(Q.qcounters + 2, (unsigned long long)(__popcll(bd) + __popcll(bd2)));
        }
    }
    if (Q.qcounters && lane == 0) {
        if (be) atomicAdd(Q.qcounters + 0, (unsigned long long)__popcll(be));
        if (bc) atomicAdd(Q.qcounters + 1, (unsigned long long)__popcll(bc));
    }
}

// The staged path of a tiled workgroup: each wave reserves its created
// particles' slots among the slice's with one LDS atomic (total: the
// slice's count, events: its event counts), writes the first kQedStage of
// the slice into its staging entries and appends any beyond with one global
// atomic each (rare: a slice makes ~1-2 particles in the monopole
// workload).  Every lane of the wave calls it.
__device__ __forceinline__ void qed_stage(const StepArgs& A, const QedArgs& Q, int64_t slice, const Created& cr,
                                          const QedEvents& qe, unsigned* total, unsigned* ev) {
    const unsigned long long b1 = __ballot(cr.n & 1), b2 = __ballot(cr.n >> 1);
    const unsigned long long be = __ballot(qe.emitted), bc = __ballot(qe.converted);
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
        if (be) atomicAdd(ev + 0, (unsigned)__popcll(be));
        if (bc) atomicAdd(ev + 1, (unsigned)__popcll(bc));
    }
    if ((b1 | b2) == 0) return;                               // wave-uniform
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned wave_total = __popcll(b1) + 2 * __popcll(b2);
    const unsigned before = __popcll(b1 & below) + 2 * __popcll(b2 & below);
    unsigned off = 0;
    if (lane == 0) off = atomicAdd(total, wave_total);
    off = __shfl(off, 0) + before;
    int dropped = 0;
    auto put = [&](unsigned k, int sp, uint64_t tag) {
        if (k < (unsigned)kQedStage) {
            const int64_t e = slice * kQedStage + k;
            Q.st.cell[e] = cr.cell;
            Q.st.xr[e] = cr.xr;
            Q.st.xth[e] = cr.xth;
            Q.st.ur[e] = cr.u[0];
            Q.st.uth[e] = cr.u[1];
            Q.st.uph[e] = cr.u[2];
            Q.st.w[e] = cr.w;
            Q.st.sp[e] = (uint8_t)sp;
            Q.st.tag[e] = tag;
            return;
        }
        const int64_t q = Q.n_used[0] + (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(Q.n_used + 1), 1ull);
        if (q >= Q.cap) {
            ++dropped;
            return;
        }
        A.cell[q] = cr.cell;
        static_cast<double*>(A.xr)[q] = cr.xr;
        static_cast<double*>(A.xth)[q] = cr.xth;
        static_cast<double*>(A.ur)[q] = cr.u[0];
        static_cast<double*>(A.uth)[q] = cr.u[1];
        static_cast<double*>(A.uph)[q] = cr.u[2];
        static_cast<double*>(A.w)[q] = cr.w;
        const_cast<uint8_t*>(A.sp)[q] = (uint8_t)sp;
        Q.tag[q] = tag;
        if (A.phi) static_cast<double*>(A.phi)[q] = 0.0;
    };
    if (cr.n >= 1) put(off, cr.sp[0], cr.tag[0]);
    if (cr.n == 2) put(off + 1, cr.sp[1], cr.tag[1]);
    if (Q.qcounters && dropped) atomicAdd(Q.qcounters + 2, (unsigned long long)dropped);
}

}  // namespace grpic
