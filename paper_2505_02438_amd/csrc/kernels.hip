// gfx950 kernels for SIMP assembly, element energies, compliance and the
// assembly backward (arXiv 2505.02438: Sec. 2.1 SIMP, Sec. 2.2 Eq. cmpd,
// Sec. 5.5 fast assembly, Appendix D sensitivity).
//
// Element matrix in separated ("fast assembly") form.  For an affine element
// with G = J^-1 (G[m][a] = d xi_m / d x_a) and the reference tensor
// M_ij[m][n] = int_ref d_m phi_i d_n phi_j, the block (i, j) of K_e^0 is
//     K_e^0(i,j) = |det J| L(A_ij),  A_ij = G^T M_ij G,
//     L(A) = lambda A + mu A^T + mu tr(A) I
// (the isotropic form lambda div u div v + 2 mu eps(u):eps(v) written per
// block; plane stress uses lambda* = E nu / (1 - nu^2)).  L is linear, so the
// assembled block is L applied to sum_e E(rho_e) |det J_e| A_ij(e): every
// element contribution costs two 3x3x3 products (T = M_ij G', A += G'^T T with
// G' = sqrt(E |det J|) G) and L is applied once per stored block.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cstdint>
#include <map>
#include <atomic>
#include <mutex>

#include "block_sum.h"
#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

// kept out of line: inlined, its polynomial constants stay resident in VGPRs
// across the callers' loops
__device__ __noinline__ double pow_general(double x, double p) { return pow(x, p); }

__device__ __forceinline__ double simp_pow(double x, double p, int ip) {
    if (ip >= 0) {
        double r = 1.0;
        for (int k = 0; k < ip; k++) r *= x;
        return r;
    }
    return pow_general(x, p);
}

template <int PREC>
__device__ __forceinline__ double load_rho(const void *rho, int64_t e) {
    if (PREC == kF64) return static_cast<const double *>(rho)[e];
    return (double)static_cast<const float *>(rho)[e];
}

template <int PREC>
__device__ __forceinline__ void store_out(void *out, int64_t e, double v) {
    if (PREC == kF64) static_cast<double *>(out)[e] = v;
    else static_cast<float *>(out)[e] = (float)v;
}

template <int PREC> struct CT { using T = float; };
template <> struct CT<kF64> { using T = double; };

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Reads of tables that no kernel writes (plan, reference tensor) through the
// constant address space: at wave-uniform indices they become scalar loads
// through the scalar cache, unaffected by the wave-level LDS fences.
template <class T>
__device__ __forceinline__ T ldc(const T *base, int64_t idx) {
    return ((const __attribute__((address_space(4))) T *)(base))[idx];
}

// c[0] = sum of partials[0:n]; c[1] = sum of partials[n:2n] (f^T u, or 0),
// by one wave, in the order of a 256-thread block: thread t adds partials t,
// t + 256, ... in turn, then the 256 sums meet in a tree (t += t + 128, then
// t + 64, ... down to t + 1).  Lane l holds threads l, l + 64, l + 128 and
// l + 192; the tree's first two levels are its own, the rest shuffles.
__device__ __forceinline__ void wave_finalize(const double *partials, int n, int with_f, double *c, int lane) {
    for (int which = 0; which < 2; which++) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        if (which == 0 || with_f) {
            // four rounds of 256 loaded together, then added in order (only
            // the terms that exist: the sums match the block's bit for bit)
            const double *src = partials + (int64_t)which * n;
            for (int k0 = lane; k0 < n; k0 += 4 * 256) {
                double x[4][4];
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int k = k0 + 64 * v + 256 * j;
                        x[j][v] = k < n ? src[k] : 0.0;
                    }
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++)
                        if (k0 + 64 * v + 256 * j < n) t[v] += x[j][v];
            }
        }
        double x = (t[0] + t[2]) + (t[1] + t[3]);
        for (int st = 32; st > 0; st >>= 1) x += __shfl_down(x, st);
        if (lane == 0) c[which] = x;
    }
}

// eight consecutive wave-uniform int32 by one scalar load
typedef int Codes8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ Codes8 ld_codes8(const int32_t *p) {
    return *((const __attribute__((address_space(4))) Codes8 *)(p));
}

}  // namespace

// ------------------------------------------------------------------ assembly
//
// acc += G'^T M_ij G' in the precision of the form (FP64 accumulation)
template <int DIM, int PREC, typename T>
__device__ __forceinline__ void accumulate(const T (&G)[DIM][DIM], const T (&M)[DIM * DIM], double (&acc)[DIM][DIM]) {
    T Tm[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; m++)
#pragma unroll
        for (int b = 0; b < DIM; b++) {
            T s = 0;
#pragma unroll
            for (int n = 0; n < DIM; n++) s += M[m * DIM + n] * G[n][b];
            Tm[m][b] = s;
        }
    if (PREC == kF64) {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++)
#pragma unroll
                for (int m = 0; m < DIM; m++) acc[a][b] += (double)G[m][a] * (double)Tm[m][b];
    } else {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++) {
                T s = 0;
#pragma unroll
                for (int m = 0; m < DIM; m++) s += G[m][a] * Tm[m][b];
                acc[a][b] += (double)s;
            }
    }
}

// G'_aa G'_cc in the form's precision
template <int PREC, typename T>
__device__ __forceinline__ T diag_product(T da, T dc) {
    if (PREC == kF64) return da * dc;
    return (T)((float)da * (float)dc);
}

// acc += G'^T M_ij G' for diagonal G': entry (a, b) is G'_aa G'_bb M_ij[a][b];
// dd holds the products G'_aa G'_bb
template <int DIM, int PREC, typename T>
__device__ __forceinline__ void accumulate_diag(const T (&dd)[DIM][DIM], const T (&M)[DIM * DIM],
                                                double (&acc)[DIM][DIM]) {
#pragma unroll
    for (int a = 0; a < DIM; a++)
#pragma unroll
        for (int b = 0; b < DIM; b++) {
            if (PREC == kF64) acc[a][b] += (double)dd[a][b] * (double)M[a * DIM + b];
            else acc[a][b] += (double)((float)dd[a][b] * (float)M[a * DIM + b]);
        }
}

static size_t assemble_lds_bytes(int dim, int nen, int prec, int64_t stage, int kmax) {
    const size_t csz = prec == kF64 ? 8 : 4;
    return 2 * 8 * (size_t)stage + 2 * csz * dim * dim * kGroupElems + csz * nen * nen * dim * dim +
           3 * kGroupNodes * 2 * 4 + 2 * 2 * (size_t)kmax * kGroupNodes;
}

// Dirichlet bits of one stored block (node n, neighbour J): bit a (a < DIM):
// row dof DIM n + a is fixed; bit 3 + c: column dof DIM J + c is fixed; bit 6:
// J == n.  An entry in a fixed row or column is 0, the diagonal entry of a
// fixed dof 1 (zero prescribed values).
__device__ __forceinline__ double dirichlet_entry(int bits, int a, int c, double v) {
    if (((bits >> a) | (bits >> (3 + c))) & 1) return (a == c && (bits & 64)) ? 1.0 : 0.0;
    return v;
}

// Geometry held per element slot of a group in LDS: G' (kGeoFull), its
// diagonal for an axis-aligned group (kGeoDiag), or for Q1 elements whose map
// is not affine the scaled physical gradients of the element's nodes at QP
// Gauss points, GEOM = kGeoPoint + QP (FP64 only)
constexpr int kGeoFull = 0, kGeoDiag = 1, kGeoPoint = 16;
// passes of the per-point form over its Gauss points: a pass after the first
// starts each block from the partial sum in the stage (kPassInit); the last
// applies L and writes the block (kPassFinal), the others write the raw sum
constexpr int kPassInit = 1, kPassFinal = 2;

// One contribution of an element slot with per-point geometry, local pair
// (i, j), added to acc when ok: sum over the QP points q of the pass, in
// order, of g_i(q) g_j(q)^T, with g_k(q) = sqrt(E w_q |det J_q|) J_q^-T grad
// phi_k(xi_q) held in Gs ([QP][NEN][DIM][kGroupElems]).  The LDS reads
// happen whether or not ok.
template <int DIM, int NEN, int QP>
__device__ __forceinline__ void contribute_point(const double *Gs, int slot, int i, int j, bool ok,
                                                 double (&acc)[DIM][DIM]) {
#pragma unroll
    for (int q = 0; q < QP; q++) {
        double gi[DIM], gj[DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            gi[a] = Gs[((q * NEN + i) * DIM + a) * kGroupElems + slot];
            gj[a] = Gs[((q * NEN + j) * DIM + a) * kGroupElems + slot];
        }
        if (ok) {
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) acc[a][c] = fma(gi[a], gj[c], acc[a][c]);
        }
    }
}

// ---- the roles' work on one group, shared by the persistent kernel
// (k_assemble), the one-workgroup-per-group kernel (k_assemble_os) and the
// per-point kernel (k_assemble_quad).  The group's data in LDS: hdr (nn,
// deg, posoff, blk, flags, first wide work item, number of wide work items,
// Dirichlet-bits offset, rank-table offset), stage (its row blocks, blk
// doubles per node), sG (the slots' geometry in the layout of GEOM), sM (the
// reference tensor, or the reference gradients at the Gauss points), sn2l
// (slot of element k of each node, [K][32]); ticket counts the group's work
// items.  GEOM is decided once per group, so the contraction loop has no
// branch on it.

// ---- compute role, wide work items (groups of at most N = 8 or 16
// nodes): lane = (pp Q + q) N + node takes position p[pp] of the item and
// its contributions q, q + Q, ...; the Q phases of a position are then
// added by a butterfly over the phase bits of the lane index (a fixed
// order), and phase 0 writes the block
template <int DIM, int NEN, int PREC, bool FUSE, int GEOM>
__device__ __forceinline__ void assemble_wide(const AsmParams &P, const int *hdr, int *ticket, double *stage,
                                              const typename CT<PREC>::T *sG, const typename CT<PREC>::T *sM,
                                              const uint16_t *sn2l, int lane, int pmode = kPassFinal) {
    using T = typename CT<PREC>::T;
    constexpr int D2 = DIM * DIM;
    constexpr int NG = kGroupNodes;
    const int nn = wave_uniform(hdr[0]);
    const int deg = wave_uniform(hdr[1]);
    const int blk = wave_uniform(hdr[3]);
    const int flags = wave_uniform(hdr[4]);
    const int wi0 = wave_uniform(hdr[5]);
    const int nwi = wave_uniform(hdr[6]);
    const int bcoff = FUSE ? wave_uniform(hdr[7]) : -1;
    const int rkoff = wave_uniform(hdr[8]);
    const int lgN = 5 - ((flags >> kGrpWideShift) & 3);  // N = 8 or 16
    const int N = 1 << lgN;
    const int rl = DIM * deg;
    const int node = lane & (N - 1);
    double *st = stage + node * blk;
    const T *G = sG;
    const uint16_t *n2l = sn2l + node;
    for (;;) {
        int r = 0;
        if (lane == 0) r = atomicAdd(ticket, 1);
        r = wave_uniform(r);
        if (r >= nwi) break;
        const int32_t *rec = P.sig_witems + (int64_t)(wi0 + r) * kWideInts;
        const int np = ldc(rec, 0), Q = ldc(rec, 1), nt = ldc(rec, 2);
        const int lgQ = 31 - __clz(Q);
        const int grp = lane >> lgN;
        const int pp = grp >> lgQ, q = grp & (Q - 1);
        // this lane's position, its contribution offset and count
        int p = -1, off = 0, cnt = 0;
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (pp == k) {
                p = ldc(rec, 8 + k);
                off = ldc(rec, 16 + k);
                cnt = ldc(rec, 24 + k);
            }
        const bool mine = pp < np && node < nn;
        // Dirichlet bits of the lane's block and its CSR position (a
        // canonical-order plan's rank table), fetched now and used at the end
        const int bcb = (FUSE && bcoff >= 0 && mine && q == 0) ? P.bc_bits[bcoff + node * deg + p] : 0;
        const int pcsr = (rkoff >= 0 && mine && q == 0) ? (int)P.grp_rank[rkoff + p * NG + node] : p;
        double acc[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) acc[a][c] = 0.0;
        if constexpr (GEOM > kGeoPoint) {
            // a later pass over the Gauss points: the block's partial sum so far
            if ((pmode & kPassInit) && mine && q == 0)
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int c = 0; c < DIM; c++) acc[a][c] = st[a * rl + DIM * pcsr + c];
        }
        // contributions of this lane: all loads first (nt <= 8)
        int pk[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int ti = q + t * Q;
            pk[t] = (t < nt && mine && ti < cnt) ? P.sig_contrib[off + ti] : -1;
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
            if (t >= nt) break;
            if (pk[t] >= 0) {
                const int k = pk[t] >> 16, i = (pk[t] >> 8) & 255, j = pk[t] & 255;
                const int slot = n2l[k * NG];
                if constexpr (GEOM > kGeoPoint) {
                    contribute_point<DIM, NEN, GEOM - kGeoPoint>(G, slot, i, j, true, acc);
                } else {
                    const T *Mij = sM + (i * NEN + j) * D2;
                    T Mv[D2];
#pragma unroll
                    for (int x = 0; x < D2; x++) Mv[x] = Mij[x];
                    if constexpr (GEOM == kGeoDiag) {
                        T dd[DIM][DIM];
#pragma unroll
                        for (int a = 0; a < DIM; a++)
#pragma unroll
                            for (int c = a; c < DIM; c++) {
                                dd[a][c] = diag_product<PREC>(G[a * kGroupElems + slot], G[c * kGroupElems + slot]);
                                dd[c][a] = dd[a][c];
                            }
                        accumulate_diag<DIM, PREC>(dd, Mv, acc);
                    } else {
                        T Gv[DIM][DIM];
#pragma unroll
                        for (int m = 0; m < DIM; m++)
#pragma unroll
                            for (int a = 0; a < DIM; a++) Gv[m][a] = G[(m * DIM + a) * kGroupElems + slot];
                        accumulate<DIM, PREC>(Gv, Mv, acc);
                    }
                }
            }
        }
        for (int sh = N; sh < N * Q; sh <<= 1)
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) acc[a][c] += __shfl_xor(acc[a][c], sh);
        if constexpr (GEOM > kGeoPoint) {
            if (!(pmode & kPassFinal)) {
                if (mine && q == 0)
#pragma unroll
                    for (int a = 0; a < DIM; a++)
#pragma unroll
                        for (int c = 0; c < DIM; c++) st[a * rl + DIM * pcsr + c] = acc[a][c];
                continue;
            }
        }
        if (mine && q == 0) {
            double tr = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; a++) tr += acc[a][a];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) {
                    double o = P.lam * acc[a][c] + P.mu * acc[c][a];
                    if (a == c) o += P.mu * tr;
                    if (FUSE && bcoff >= 0) o = dirichlet_entry(bcb, a, c, o);
                    st[a * rl + DIM * pcsr + c] = o;
                }
        }
    }
}

// compute role, work items of position pairs (groups of up to 32 nodes)
template <int DIM, int NEN, int PREC, bool FUSE, int GEOM>
__device__ __forceinline__ void assemble_pairs(const AsmParams &P, const int *hdr, int *ticket, double *stage,
                                               const typename CT<PREC>::T *sG, const typename CT<PREC>::T *sM,
                                               const uint16_t *sn2l, int lane, int pmode = kPassFinal) {
    using T = typename CT<PREC>::T;
    constexpr int D2 = DIM * DIM;
    constexpr int NG = kGroupNodes;
    const int nn = wave_uniform(hdr[0]);
    const int deg = wave_uniform(hdr[1]);
    const int posoff = wave_uniform(hdr[2]);
    const int blk = wave_uniform(hdr[3]);
    const int bcoff = FUSE ? wave_uniform(hdr[7]) : -1;
    const int rkoff = wave_uniform(hdr[8]);
    const int rl = DIM * deg;
    const bool hi = lane >= NG;
    const int node = lane & (NG - 1);
    double *st = stage + node * blk;
    const T *G = sG;
    const uint16_t *n2l = sn2l + node;
    for (;;) {
        int r = 0;
        if (lane == 0) r = atomicAdd(ticket, 1);
        r = wave_uniform(r);
        // the signature's slice holds deg + 1 items, the last ones -1;
        // late waves draw tickets past the end
        if (r > deg) break;
        const int pa = ldc(P.sig_pairs, 2 * posoff + 2 * r);
        if (pa < 0) break;
        const int pb = ldc(P.sig_pairs, 2 * posoff + 2 * r + 1);
        const bool split = pb == pa;
        const int c0 = ldc(P.sig_pos_ptr, posoff + pa);
        const int na = ldc(P.sig_pos_ptr, posoff + pa + 1) - c0;
        // contribution ranges of the two halves: [lo0, lo0 + nlo), [hi0, hi0 + nhi)
        int lo0 = c0, nlo = na, hi0 = c0, nhi = 0;
        if (split) {
            nlo = (na + 1) / 2;
            hi0 = c0 + nlo;
            nhi = na - nlo;
        } else if (pb >= 0) {
            hi0 = ldc(P.sig_pos_ptr, posoff + pb);
            nhi = ldc(P.sig_pos_ptr, posoff + pb + 1) - hi0;
        }
        const int mycnt = hi ? nhi : nlo;
        // Dirichlet bits of the lane's block, fetched now and used at the end
        const int pme = hi ? pb : pa;
        const int bcb = (FUSE && bcoff >= 0 && node < nn && pme >= 0) ? P.bc_bits[bcoff + node * deg + pme] : 0;
        // the block's CSR position (a canonical-order plan's rank table)
        const int pcsr = (rkoff >= 0 && node < nn && pme >= 0) ? (int)P.grp_rank[rkoff + pme * NG + node] : pme;
        double acc[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) acc[a][c] = 0.0;
        if constexpr (GEOM > kGeoPoint) {
            // a later pass over the Gauss points: the block's partial sum so
            // far, in the lane that writes the block
            if ((pmode & kPassInit) && node < nn && pme >= 0 && !(split && hi))
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int c = 0; c < DIM; c++) acc[a][c] = st[a * rl + DIM * pcsr + c];
        }
        // nlo >= nhi: the low half has the longer list.  The codes of a chunk
        // of 8 contributions of each half are read by scalar loads before the
        // chunk's LDS reads (scalar loads and LDS reads share one wait
        // counter: a scalar load waited for between contributions would also
        // wait for every LDS read in flight).  Both halves read as many
        // chunks as the longer list needs, past a list's end into the next
        // codes (the table ends with enough zero codes); such entries are
        // read but not added.
        const int32_t *lo_p = P.sig_contrib + lo0;
        const int32_t *hi_p = P.sig_contrib + (nhi > 0 ? hi0 : lo0);
        for (int t0 = 0; t0 < nlo; t0 += 8) {
            const Codes8 cl = ld_codes8(lo_p + t0), ch = ld_codes8(hi_p + t0);
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (t0 + u >= nlo) break;
                // an entry past the lane's own (shorter) list reads with
                // code 0, a slot of its own table, and is not added
                const bool oku = t0 + u < mycnt;
                const int code = oku ? (hi && nhi > 0 ? ch[u] : cl[u]) : 0;
                const int k = code >> 16, i = (code >> 8) & 255, j = code & 255;
                const int slot = n2l[k * NG];
                if constexpr (GEOM > kGeoPoint) {
                    contribute_point<DIM, NEN, GEOM - kGeoPoint>(G, slot, i, j, oku, acc);
                } else {
                    const T *Mij = sM + (i * NEN + j) * D2;
                    T Mv[D2];
#pragma unroll
                    for (int x = 0; x < D2; x++) Mv[x] = Mij[x];
                    if constexpr (GEOM == kGeoDiag) {
                        T dd[DIM][DIM];
#pragma unroll
                        for (int a = 0; a < DIM; a++)
#pragma unroll
                            for (int c = a; c < DIM; c++) {
                                dd[a][c] = diag_product<PREC>(G[a * kGroupElems + slot], G[c * kGroupElems + slot]);
                                dd[c][a] = dd[a][c];
                            }
                        if (oku) accumulate_diag<DIM, PREC>(dd, Mv, acc);
                    } else {
                        T Gv[DIM][DIM];
#pragma unroll
                        for (int m = 0; m < DIM; m++)
#pragma unroll
                            for (int a = 0; a < DIM; a++) Gv[m][a] = G[(m * DIM + a) * kGroupElems + slot];
                        if (oku) accumulate<DIM, PREC>(Gv, Mv, acc);
                    }
                }
            }
        }
        if (split) {
            // low half's sum + high half's sum (the same in both halves:
            // addition is commutative)
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) acc[a][c] += __shfl_xor(acc[a][c], NG);
        }
        if constexpr (GEOM > kGeoPoint) {
            if (!(pmode & kPassFinal)) {
                if (node < nn && pme >= 0 && !(split && hi))
#pragma unroll
                    for (int a = 0; a < DIM; a++)
#pragma unroll
                        for (int c = 0; c < DIM; c++) st[a * rl + DIM * pcsr + c] = acc[a][c];
                continue;
            }
        }
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; a++) tr += acc[a][a];
        const int p = hi ? pb : pa;
        if (node < nn && p >= 0 && !(split && hi)) {
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) {
                    double o = P.lam * acc[a][c] + P.mu * acc[c][a];
                    if (a == c) o += P.mu * tr;
                    if (FUSE && bcoff >= 0) o = dirichlet_entry(bcb, a, c, o);
                    st[a * rl + DIM * pcsr + c] = o;
                }
        }
    }
}

// compute role of one group: wide or paired work items; only Q1 elements
// (quadrilaterals, hexahedra) can form axis-aligned groups
template <int DIM, int NEN, int PREC, bool FUSE>
__device__ __forceinline__ void assemble_group(const AsmParams &P, const int *hdr, int *ticket, double *stage,
                                               const typename CT<PREC>::T *sG, const typename CT<PREC>::T *sM,
                                               const uint16_t *sn2l, int lane) {
    constexpr bool kMayDiag = NEN == (1 << DIM);
    const int flags = wave_uniform(hdr[4]);
    const bool diag = kMayDiag && (flags & kGrpDiag);
    constexpr int kDiag = kMayDiag ? kGeoDiag : kGeoFull;
    if (flags >> kGrpWideShift) {
        if (diag) assemble_wide<DIM, NEN, PREC, FUSE, kDiag>(P, hdr, ticket, stage, sG, sM, sn2l, lane);
        else assemble_wide<DIM, NEN, PREC, FUSE, kGeoFull>(P, hdr, ticket, stage, sG, sM, sn2l, lane);
    } else {
        if (diag) assemble_pairs<DIM, NEN, PREC, FUSE, kDiag>(P, hdr, ticket, stage, sG, sM, sn2l, lane);
        else assemble_pairs<DIM, NEN, PREC, FUSE, kGeoFull>(P, hdr, ticket, stage, sG, sM, sn2l, lane);
    }
}

// ---- store role: one group's stage sb with its row offsets rows, as store
// wave sw of KSTORE.  Each store wave takes every KSTORE-th node of the
// group's first half together with its partner half a group later, four
// values per lane and node at a time, so that eight LDS reads are in flight
// per batch.  K is
// written once and never read back here: the stores are non-temporal, so
// they stream out instead of taking L2 lines that the element loads use
template <int DIM, int KSTORE>
__device__ __forceinline__ void store_rows(const AsmParams &P, const int *hdr, const int32_t *rows, const double *sb,
                                           int sw, int lane) {
    const int nn = wave_uniform(hdr[0]);
    const int deg = wave_uniform(hdr[1]);
    const int blk = wave_uniform(hdr[3]);
    const int bsz = DIM * DIM * deg;  // the node's DIM rows, contiguous in CSR
    if (DIM == 2 && bsz <= 64) {
        // short row blocks (2D elements): lane = (node j of npi, value o),
        // so that one batch of four stores covers 4 npi of the wave's
        // nodes w', w' + KSTORE, ... instead of one node per store
        const int npi = 64 / bsz;  // nodes per store instruction
        const int j = lane / bsz, o = lane - j * bsz;
        for (int b0 = 0; b0 * KSTORE + sw < nn; b0 += 4 * npi) {
            double v[4];
            int dst[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int n = sw + KSTORE * (b0 + c * npi + j);
                const bool ok = j < npi && n < nn;
                v[c] = ok ? sb[n * blk + o] : 0.0;
                dst[c] = ok ? rows[2 * n] + o : -1;
            }
#pragma unroll
            for (int c = 0; c < 4; c++)
                if (dst[c] >= 0) __builtin_nontemporal_store(v[c], P.K + dst[c]);
        }
        return;
    }
    // a wave's two nodes of a batch lie half a group apart
    const int half = (nn + 1) / 2;
    if (wave_uniform(hdr[8]) >= 0) {
        // the group's nodes are scattered over K (a plan in canonical order,
        // with a rank table): each node's run is issued from the 128 B line
        // boundary at or below its start (lanes before the start or past the
        // end store nothing), so that a store instruction covers whole lines
        // and only a run's first and last lines are written in part.  Runs
        // of consecutive nodes (below) are issued from their starts instead:
        // the neighbouring runs complete the lines they share while both are
        // in the cache, and the shorter code keeps the store waves' issue
        // rate up
        for (int n0 = sw; n0 < half; n0 += KSTORE) {
            const int n1 = n0 + half;
            const bool two = n1 < nn;
            const int base0 = wave_uniform(rows[2 * n0]);
            const int base1 = two ? wave_uniform(rows[2 * n1]) : base0;
            const int sh0 = base0 & 15, sh1 = base1 & 15;
            const double *s0 = sb + n0 * blk;
            const double *s1 = sb + (two ? n1 : n0) * blk;
            const int span = bsz + (sh0 > sh1 ? sh0 : sh1);
            for (int c0 = 0; c0 < span; c0 += 4 * 64) {
                double v0[4], v1[4];
                bool k0[4], k1[4];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const int q0 = c0 + 64 * c + lane - sh0, q1 = c0 + 64 * c + lane - sh1;
                    k0[c] = q0 >= 0 && q0 < bsz;
                    k1[c] = two && q1 >= 0 && q1 < bsz;
                    v0[c] = k0[c] ? s0[q0] : 0.0;
                    v1[c] = k1[c] ? s1[q1] : 0.0;
                }
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    if (k0[c]) __builtin_nontemporal_store(v0[c], P.K + base0 + (c0 + 64 * c + lane - sh0));
                    if (k1[c]) __builtin_nontemporal_store(v1[c], P.K + base1 + (c0 + 64 * c + lane - sh1));
                }
            }
        }
        return;
    }
    for (int n0 = sw; n0 < half; n0 += KSTORE) {
        const int n1 = n0 + half;
        const bool two = n1 < nn;
        const int base0 = rows[2 * n0];
        const int base1 = two ? rows[2 * n1] : base0;
        const double *s0 = sb + n0 * blk;
        const double *s1 = sb + (two ? n1 : n0) * blk;
        for (int o0 = lane; o0 < bsz; o0 += 4 * 64) {
            double v0[4], v1[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int o = o0 + 64 * c;
                v0[c] = o < bsz ? s0[o] : 0.0;
                v1[c] = o < bsz ? s1[o] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int o = o0 + 64 * c;
                if (o < bsz) {
                    __builtin_nontemporal_store(v0[c], P.K + base0 + o);
                    if (two) __builtin_nontemporal_store(v1[c], P.K + base1 + o);
                }
            }
        }
    }
}

// Persistent, warp-specialised assembly.  One workgroup of 16 waves per CU
// walks the node groups g0 = blockIdx.x, g0 + gridDim.x, ...  The groups are
// in node order, so at any time the whole chip writes one contiguous stretch
// of K (a window of gridDim.x consecutive groups).  Workgroups are dealt to
// the 8 XCDs round robin; workgroup b takes slot (b mod 8) gridDim.x/8 + b/8
// of each window, so every XCD walks a contiguous run of the window and
// neighbouring groups find their shared element data in that XCD's L2
// (slicing the whole group range per XCD instead spreads the writes over
// eight distant stretches and is slower).
// In step s:
//   - compute waves (0..7) assemble group s into LDS stage s&1: each takes a
//     pair of neighbour positions of the group's signature from a ticket
//     (costliest first); the low half of the wave walks the first position's
//     contributions, the high half the second's, lane = node of the group;
//     a finished DIM x DIM block goes to the node's row block in the stage;
//   - store waves (8..11) write group s-1 from stage (s-1)&1: every node's
//     DIM rows are contiguous in CSR and go out as one run.  They issue
//     stores only and never wait for them, so the CU's stores stream while
//     the next groups are computed;
//   - load waves (12..15) load group s+1 (G' = sqrt(E(rho) det J) J^-1, or
//     for an axis-aligned group its diagonal G'_aa, the slot table and the
//     row offsets) into the other LDS buffers.  They load only, so their
//     waits cover their own loads and none of the stores.
// One workgroup barrier ends a step.  Summation order of a stored block: the
// signature's contribution order (ascending element within the block; for a
// wide work item, each phase's contributions in that order, then the phases
// by a butterfly), then L(A) = lam A + mu A^T + mu tr(A) I; fixed by the
// mesh, independent of waves and streams.
//
// FUSE (soptx_step): the compute waves also apply a bound Dirichlet table
// while they stage a block (a fixed row or column: 0, the diagonal entry of a
// fixed dof: 1), so the stored K already carries the boundary conditions and
// no pass of its own follows.

constexpr int kAsmThreads = 1024;
constexpr int kLoadWaves = 4;
// compute and store waves of the persistent kernel (with the 4 load waves, 16
// in all): P2 tetrahedra, whose steps are paced by the compute waves, take
// two waves from the store role
template <int NEN>
struct Roles {
    static constexpr int comp = NEN == 10 ? 10 : 8;
    static constexpr int store = kAsmThreads / 64 - kLoadWaves - comp;
};
static_assert(2 * kGroupNodes == 64, "two positions per wavefront");

template <int DIM, int NEN, int PREC, bool FUSE>
__global__ __launch_bounds__(kAsmThreads, 1) void k_assemble(AsmParams P) {
    using T = typename CT<PREC>::T;
    using R = typename std::conditional<PREC == kF64, double, float>::type;  // rho as stored
    constexpr int D2 = DIM * DIM;
    constexpr int NG = kGroupNodes;
    constexpr int kCompWaves = Roles<NEN>::comp, kStoreWaves = Roles<NEN>::store;
    constexpr int kLoadBase = (kCompWaves + kStoreWaves) * 64;
    constexpr int kSetThreads = kLoadWaves / 2 * 64;  // threads of one load set
    constexpr int NPF = (kMaxAdjacent * NG + kSetThreads - 1) / kSetThreads;  // slot entries per load thread
    static_assert(kGroupElems <= 2 * kSetThreads, "two elements per load thread");
    static_assert(2 * NG <= kSetThreads, "row offsets: one per load thread");
    extern __shared__ __align__(16) unsigned char smem[];
    double *stage = reinterpret_cast<double *>(smem);                      // [2][P.stage]
    T *sG = reinterpret_cast<T *>(stage + 2 * P.stage);                     // [2][D2][kGroupElems]
    T *sM = sG + 2 * D2 * kGroupElems;                                      // [NEN][NEN][D2]
    int32_t *srows = reinterpret_cast<int32_t *>(sM + NEN * NEN * D2);      // [3][NG][2]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(srows + 3 * NG * 2);      // [2][kmax][NG]
    __shared__ int ticket[2];
    // group headers, one per row-offset buffer: nn, deg, posoff, blk, flags,
    // first wide work item, number of wide work items, offset of the group's
    // Dirichlet bits (-1: none), offset of its rank table (-1: none).
    // Written by the load waves with the group's other data, so that the
    // compute and store waves start a step without a chain of scalar loads
    __shared__ int shdr[3][9];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int64_t NC = P.n_cells;
    const int ngr = P.n_groups;
    const int stride = gridDim.x;
    const int g0 = stride % 8 == 0 ? (int)(blockIdx.x % 8) * (stride / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    if (g0 >= ngr) return;
    const int nsteps = (ngr - 1 - g0) / stride + 2;  // groups of this workgroup, plus the last store step
    const int n2l_stride = P.kmax * NG;

    for (int x = tid; x < NEN * NEN * D2; x += kAsmThreads) {
        if (PREC == kF64) sM[x] = (T)P.M[x];
        else sM[x] = (T)P.M32[x];
    }

    // ---- load role: two sets of kLoadWaves / 2 waves; set x puts the groups
    // of the steps of parity x and has two steps to bring each one in.  A
    // thread handles elements lt and lt + kSetThreads of the group
    const int lt = (tid - kLoadBase) & (kSetThreads - 1);
    const int lset = (tid - kLoadBase) / kSetThreads;
    struct Ids {
        int e[2];
    };
    auto elem_id = [&](int gg) {
        Ids r;
        r.e[0] = r.e[1] = -1;
        if (gg < ngr) {
            const int eoff = ldc(P.grp_info, kGrpInfo * gg + 2);
            const int ne = ldc(P.grp_info, kGrpInfo * gg + 3);
#pragma unroll
            for (int h = 0; h < 2; h++)
                if (lt + h * kSetThreads < ne) r.e[h] = P.grp_elems[eoff + lt + h * kSetThreads];
        }
        return r;
    };
    struct LoadRegs {
        double pd[2][D2 + 1];
        R prho[2];
        int pn2l[NPF];
        int prow;
    };
    auto issue = [&](LoadRegs &q, int gg, const Ids &id) {
        const int sg = ldc(P.grp_info, kGrpInfo * gg + 0);
        const int off = ldc(P.grp_info, kGrpInfo * gg + 4);
        const bool diag = ldc(P.grp_info, kGrpInfo * gg + 5) & kGrpDiag;
        const int nk = ldc(P.sig_info, 4 * sg + 0) * NG;
#pragma unroll
        for (int h = 0; h < 2; h++)
            if (id.e[h] >= 0) {
                if (diag) {
                    // axis-aligned: the diagonal of J^-1 and det J
#pragma unroll
                    for (int a = 0; a < DIM; a++) q.pd[h][a * DIM + a] = P.geo[(int64_t)(a * DIM + a) * NC + id.e[h]];
                    q.pd[h][D2] = P.geo[(int64_t)D2 * NC + id.e[h]];
                } else {
#pragma unroll
                    for (int c = 0; c <= D2; c++) q.pd[h][c] = P.geo[(int64_t)c * NC + id.e[h]];
                }
                // a canonical-order plan's slots are ranks: the density is
                // read through the rank -> element map
                const int er = P.elem_by_rank ? P.elem_by_rank[id.e[h]] : id.e[h];
                q.prho[h] = static_cast<const R *>(P.rho)[er];
            }
#pragma unroll
        for (int r = 0; r < NPF; r++)
            q.pn2l[r] = lt + r * kSetThreads < nk ? P.grp_n2l[off + lt + r * kSetThreads] : 0;
        q.prow = lt < 2 * NG ? P.grp_rows[(int64_t)gg * 2 * NG + lt] : 0;
    };
    auto put = [&](const LoadRegs &q, int gg, int b, int rb) {
        const int ne = ldc(P.grp_info, kGrpInfo * gg + 3);
        const int flags = ldc(P.grp_info, kGrpInfo * gg + 5);
        const int sg = ldc(P.grp_info, kGrpInfo * gg + 0);
        const int nk = ldc(P.sig_info, 4 * sg + 0) * NG;
        T *G = sG + b * D2 * kGroupElems;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int slot = lt + h * kSetThreads;
            if (slot < ne) {
                const double E = P.Emin + simp_pow((double)q.prho[h], P.p, P.ip) * (P.E0 - P.Emin);
                const double qq = sqrt(E * q.pd[h][D2]);
                if (flags & kGrpDiag) {
                    // the diagonal G'_aa only; the compute waves form the
                    // products G'_aa G'_cc
#pragma unroll
                    for (int a = 0; a < DIM; a++) G[a * kGroupElems + slot] = (T)(qq * q.pd[h][a * DIM + a]);
                } else {
#pragma unroll
                    for (int c = 0; c < D2; c++) G[c * kGroupElems + slot] = (T)(qq * q.pd[h][c]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NPF; r++)
            if (lt + r * kSetThreads < nk) sn2l[b * n2l_stride + lt + r * kSetThreads] = (uint16_t)q.pn2l[r];
        if (lt < 2 * NG) srows[rb * 2 * NG + lt] = q.prow;
        if (lt == 0) {
            ticket[b] = 0;
            shdr[rb][0] = ldc(P.grp_info, kGrpInfo * gg + 1);
            shdr[rb][1] = ldc(P.sig_info, 4 * sg + 1);
            shdr[rb][2] = ldc(P.sig_info, 4 * sg + 2);
            shdr[rb][3] = ldc(P.sig_info, 4 * sg + 3);
            shdr[rb][4] = flags;
            const int wi0 = ldc(P.sig_witem_ptr, sg);
            shdr[rb][5] = wi0;
            shdr[rb][6] = ldc(P.sig_witem_ptr, sg + 1) - wi0;
            shdr[rb][7] = (FUSE && P.bc_off) ? P.bc_off[gg] : -1;
            shdr[rb][8] = P.grp_rank_off ? P.grp_rank_off[gg] : -1;
        }
    };

    auto compute_group = [&](int b, int rb) {
        assemble_group<DIM, NEN, PREC, FUSE>(P, shdr[rb], &ticket[b], stage + b * P.stage, sG + b * D2 * kGroupElems, sM,
                                             sn2l + b * n2l_stride, lane);
    };
    auto store_group = [&](int b, int rb) {
        store_rows<DIM, kStoreWaves>(P, shdr[rb], srows + rb * 2 * NG, stage + b * P.stage, w - kCompWaves, lane);
    };

    // Every wave runs nsteps + 1 barriers: one after the prologue, one per
    // step.  The roles run separate loops so that a load in flight across a
    // barrier on a load wave is no wait on another role's path.
    if (w < kCompWaves) {
        __syncthreads();
        for (int s = 0; s < nsteps; s++) {
            const int g = g0 + s * stride;
            if (g < ngr) compute_group(s & 1, s % 3);
            __syncthreads();
        }
    } else if (w < kCompWaves + kStoreWaves) {
        __syncthreads();
        for (int s = 0; s < nsteps; s++) {
            if (s > 0) store_group((s - 1) & 1, (s - 1) % 3);
            // step 0 has nothing to store: the first store wave of workgroup
            // 0 adds the energy kernel's partials of c there
            else if (P.fin_c && blockIdx.x == 0 && w == kCompWaves)
                wave_finalize(P.fin_partials, P.fin_n, P.fin_with_f, P.fin_c, lane);
            __syncthreads();
        }
    } else {
        // group k stands for g0 + k stride.  Set 1 puts group 0 now; at step
        // s, set s & 1 puts group s + 1 (loaded at step s - 2, or before the
        // first barrier), issues the loads of group s + 3 and the element ids
        // of group s + 5; the other set only meets the barrier
        auto grp = [&](int k) { return g0 + k * stride; };
        // the load waves' few loads go ahead of the store waves' stream
        __builtin_amdgcn_s_setprio(3);
        LoadRegs q;
        Ids id;
        if (lset == 1) {
            const Ids i0 = elem_id(grp(0));
            issue(q, grp(0), i0);
            put(q, grp(0), 0, 0);
        }
        const int k1 = lset == 0 ? 1 : 2;  // first group this set brings in
        if (grp(k1) < ngr) issue(q, grp(k1), elem_id(grp(k1)));
        id = elem_id(grp(k1 + 2));
        __syncthreads();
        for (int s = 0; s < nsteps; s++) {
            if ((s & 1) == lset && grp(s + 1) < ngr) {
                put(q, grp(s + 1), (s + 1) & 1, (s + 1) % 3);
                if (grp(s + 3) < ngr) issue(q, grp(s + 3), id);
                id = elem_id(grp(s + 5));
            }
            __syncthreads();
        }
    }
}

// One-shot assembly: one workgroup per group (two waves in 2D, eight in 3D;
// XCD-local runs of consecutive groups inside windows of os_window
// workgroups), several workgroups per CU.  Each loads its group (element
// data, slot table, row offsets), assembles its blocks into one LDS stage
// (all its waves take work items from the ticket), then streams the stage to
// K with non-temporal stores; the hardware overlaps one workgroup's loads and
// compute with another's stores.  The blocks, their summation order and the
// stores are those of k_assemble.
template <int DIM>
struct OsShape { static constexpr int threads = DIM == 2 ? 128 : 512; };

template <int DIM, int NEN, int PREC, bool FUSE>
__global__ __launch_bounds__(OsShape<DIM>::threads) void k_assemble_os(AsmParams P) {
    constexpr int kOsThreads = OsShape<DIM>::threads;
    using T = typename CT<PREC>::T;
    using R = typename std::conditional<PREC == kF64, double, float>::type;  // rho as stored
    constexpr int D2 = DIM * DIM;
    constexpr int NG = kGroupNodes;
    constexpr int kStoreWaves = kOsThreads / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    double *stage = reinterpret_cast<double *>(smem);                  // [P.stage]
    T *sG = reinterpret_cast<T *>(stage + P.stage);                     // [D2][kGroupElems]
    T *sM = sG + D2 * kGroupElems;                                      // [NEN][NEN][D2]
    int32_t *srows = reinterpret_cast<int32_t *>(sM + NEN * NEN * D2);  // [NG][2]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(srows + NG * 2);      // [kmax][NG]
    __shared__ int ticket;
    __shared__ int shdr[9];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int64_t NC = P.n_cells;
    const int ngr = P.n_groups;
    const int W = P.os_window;
    const int bid = blockIdx.x;
    // the fused step: the first wave of workgroup 0 adds the energy kernel's
    // partials of c first
    if (P.fin_c && bid == 0 && w == 0) wave_finalize(P.fin_partials, P.fin_n, P.fin_with_f, P.fin_c, lane);
    const int base = bid - bid % W;
    const int gg = base + W <= ngr ? base + (bid % 8) * (W / 8) + (bid - base) / 8 : bid;
    if (gg >= ngr) return;
    // ---- loads
    const int sg = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 0));
    const int eoff = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 2));
    const int ne = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 3));
    const int n2off = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 4));
    const int gflags = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 5));
    const int nk = wave_uniform(ldc(P.sig_info, 4 * sg + 0)) * NG;
    for (int x = tid; x < NEN * NEN * D2; x += kOsThreads) {
        if (PREC == kF64) sM[x] = (T)P.M[x];
        else sM[x] = (T)P.M32[x];
    }
    // two slots per thread and pass, their loads in flight together (a group
    // can hold a few more elements than the workgroup has threads)
    for (int s0 = tid; s0 < ne; s0 += 2 * kOsThreads) {
        int e[2];
        double rr[2], gd[2][D2 + 1];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int slot = s0 + h * kOsThreads;
            e[h] = slot < ne ? P.grp_elems[eoff + slot] : -1;
        }
#pragma unroll
        for (int h = 0; h < 2; h++)
            if (e[h] >= 0) {
                const int eo = P.elem_by_rank ? P.elem_by_rank[e[h]] : e[h];
                rr[h] = (double)static_cast<const R *>(P.rho)[eo];
                gd[h][D2] = P.geo[(int64_t)D2 * NC + e[h]];
                if (gflags & kGrpDiag) {
#pragma unroll
                    for (int a = 0; a < DIM; a++) gd[h][a * DIM + a] = P.geo[(int64_t)(a * DIM + a) * NC + e[h]];
                } else {
#pragma unroll
                    for (int c = 0; c < D2; c++) gd[h][c] = P.geo[(int64_t)c * NC + e[h]];
                }
            }
#pragma unroll
        for (int h = 0; h < 2; h++)
            if (e[h] >= 0) {
                const int slot = s0 + h * kOsThreads;
                const double E = P.Emin + simp_pow(rr[h], P.p, P.ip) * (P.E0 - P.Emin);
                const double qq = sqrt(E * gd[h][D2]);
                if (gflags & kGrpDiag) {
#pragma unroll
                    for (int a = 0; a < DIM; a++) sG[a * kGroupElems + slot] = (T)(qq * gd[h][a * DIM + a]);
                } else {
#pragma unroll
                    for (int c = 0; c < D2; c++) sG[c * kGroupElems + slot] = (T)(qq * gd[h][c]);
                }
            }
    }
    for (int x = tid; x < nk; x += kOsThreads) sn2l[x] = P.grp_n2l[n2off + x];
    if (tid < 2 * NG) srows[tid] = P.grp_rows[(int64_t)gg * 2 * NG + tid];
    if (tid == 0) {
        ticket = 0;
        shdr[0] = ldc(P.grp_info, kGrpInfo * gg + 1);
        shdr[1] = ldc(P.sig_info, 4 * sg + 1);
        shdr[2] = ldc(P.sig_info, 4 * sg + 2);
        shdr[3] = ldc(P.sig_info, 4 * sg + 3);
        shdr[4] = gflags;
        const int wi0 = ldc(P.sig_witem_ptr, sg);
        shdr[5] = wi0;
        shdr[6] = ldc(P.sig_witem_ptr, sg + 1) - wi0;
        shdr[7] = (FUSE && P.bc_off) ? P.bc_off[gg] : -1;
        shdr[8] = P.grp_rank_off ? P.grp_rank_off[gg] : -1;
    }
    __syncthreads();

    assemble_group<DIM, NEN, PREC, FUSE>(P, shdr, &ticket, stage, sG, sM, sn2l, lane);
    __syncthreads();
    store_rows<DIM, kStoreWaves>(P, shdr, srows, stage, w, lane);
}

// Gauss points and reference gradients of Q1 elements on [0, 1]^DIM with the
// 2-point rule per axis: point q has coordinate xi_m = gp if bit m of q is
// set, else gm (gp, gm = (1 +- 1/sqrt(3)) / 2, weights 1 / 2^DIM); node k
// sits at corner bits q1_corner(k) (bit m: coordinate m): quadrilateral
// (0,0) (1,0) (1,1) (0,1), the
// hexahedron's bottom face in that order then its top face.  d phi_k / d xi_m
// = s_km prod_{n != m} (xi_n if bit n of k else 1 - xi_n), s_km = +1 if bit m
// of k else -1; the factor for axis n is gp where the bits of k and q agree
// on n, gm where they differ.
__host__ __device__ constexpr int q1_corner(int k) { return k ^ ((k >> 1) & 1); }
constexpr double kQ1Gp = 0.78867513459481288225457439025098;
constexpr double kQ1Gm = 0.21132486540518711774542560974902;

// Assembly of Q1 elements whose map is not affine, where the element matrix
// is K_e^0(i,j) = sum_q w_q |det J_q| L(g_i g_j^T) with g = J_q^-T grad phi
// at each Gauss point q.  One workgroup per node group of the same plan as
// k_assemble: the signatures' work items, the element order of the
// contributions, the stage and the row stores are the same.  An element
// slot's geometry is, per Gauss point, g_k(q) = sqrt(E(rho)) G'_q^T grad
// phi_k(xi_q) for its NEN nodes, with G'_q = sqrt(w_q |det J_q|) J_q^-1 read
// from qgeo (the per-mesh part), so a contribution is sum_q g_i(q) g_j(q)^T.
// The points are taken QP at a time (LDS holds the gradients of QP points):
// each pass forms the gradients of its points for every slot, then adds its
// points' terms of every contribution to the block's sum in the stage; the
// last pass applies L.  A block's sum: the passes in order; in a pass, the
// contributions in the plan's order, each over the pass's points in order.
// No element matrix is written to memory.  FP64; Dirichlet rows and columns
// are applied by k_dirichlet afterwards.
template <int DIM>
struct QuadShape {
    static constexpr int threads = DIM == 2 ? 256 : 1024;
    static constexpr int qp = DIM == 2 ? 4 : 3;  // Gauss points per pass
};

template <int DIM, int NEN>
__global__ __launch_bounds__(QuadShape<DIM>::threads) void k_assemble_quad(AsmParams P) {
    constexpr int kThreads = QuadShape<DIM>::threads;
    constexpr int QP = QuadShape<DIM>::qp;
    constexpr int D2 = DIM * DIM;
    constexpr int NQ = 1 << DIM;
    constexpr int NPASS = (NQ + QP - 1) / QP;
    constexpr int QLAST = NQ - (NPASS - 1) * QP;  // points of the last pass
    constexpr int NG = kGroupNodes;
    constexpr int kStoreWaves = kThreads / 64;
    static_assert(NEN == NQ, "Q1 elements");
    static_assert(kGroupElems <= kThreads, "one thread per slot");
    extern __shared__ __align__(16) unsigned char smem[];
    double *stage = reinterpret_cast<double *>(smem);               // [P.stage]
    double *sg = stage + P.stage;                                                         // [QP][NEN][DIM][kGroupElems]
    int32_t *srows = reinterpret_cast<int32_t *>(sg + QP * NEN * DIM * kGroupElems);     // [NG][2]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(srows + NG * 2);  // [kmax][NG]
    __shared__ int ticket;
    __shared__ int shdr[9];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int64_t NC = P.n_cells;
    const int ngr = P.n_groups;
    const int W = P.os_window;
    const int bid = blockIdx.x;
    const int base = bid - bid % W;
    const int gg = base + W <= ngr ? base + (bid % 8) * (W / 8) + (bid - base) / 8 : bid;
    if (gg >= ngr) return;
    const int sg_ = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 0));
    const int eoff = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 2));
    const int ne = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 3));
    const int n2off = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 4));
    const int gflags = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 5));
    const int nk = wave_uniform(ldc(P.sig_info, 4 * sg_ + 0)) * NG;
    for (int x = tid; x < nk; x += kThreads) sn2l[x] = P.grp_n2l[n2off + x];
    if (tid < 2 * NG) srows[tid] = P.grp_rows[(int64_t)gg * 2 * NG + tid];
    if (tid == 0) {
        shdr[0] = ldc(P.grp_info, kGrpInfo * gg + 1);
        shdr[1] = ldc(P.sig_info, 4 * sg_ + 1);
        shdr[2] = ldc(P.sig_info, 4 * sg_ + 2);
        shdr[3] = ldc(P.sig_info, 4 * sg_ + 3);
        shdr[4] = gflags;
        const int wi0 = ldc(P.sig_witem_ptr, sg_);
        shdr[5] = wi0;
        shdr[6] = ldc(P.sig_witem_ptr, sg_ + 1) - wi0;
        shdr[7] = -1;
        shdr[8] = P.grp_rank_off ? P.grp_rank_off[gg] : -1;
    }
    // The slots' per-point geometry is read all at once, so that one memory
    // latency covers every pass: item x = q ne + slot, thread tid takes items
    // x = NQ ne - 1 - tid - h kThreads (h = 0, 1, ...), from the last point
    // down.  Item h = 0 stays in registers until its point's pass; items h >
    // 0 exist where a group has more than kThreads / NQ slots, belong to the
    // first pass (kThreads >= (NQ - QP) kGroupElems) and are turned into
    // gradients at once.
    static_assert(kThreads >= (NQ - QP) * kGroupElems, "items past the first belong to the first pass");
    constexpr int kItems = (NQ * kGroupElems + kThreads - 1) / kThreads;
    double G[kItems][D2], se[kItems];
    int iq[kItems], islot[kItems];
#pragma unroll
    for (int h = 0; h < kItems; h++) {
        const int x = NQ * ne - 1 - tid - h * kThreads;
        iq[h] = ne > 0 && x >= 0 ? x / ne : NQ;  // NQ: no item
        islot[h] = iq[h] < NQ ? x - iq[h] * ne : 0;
        se[h] = 0.0;
        if (iq[h] < NQ) {
            const int id = P.grp_elems[eoff + islot[h]];
            const int eo = P.elem_by_rank ? P.elem_by_rank[id] : id;
            se[h] = sqrt(P.Emin + simp_pow(static_cast<const double *>(P.rho)[eo], P.p, P.ip) * (P.E0 - P.Emin));
#pragma unroll
            for (int c = 0; c < D2; c++) G[h][c] = P.qgeo[(int64_t)(iq[h] * D2 + c) * NC + id];
        }
    }
    // sg[point qq of the pass][node k][a][slot] = g_k[a] = sqrt(E) sum_m
    // grad phi_k(xi_q)[m] G'_q[m][a]
    auto gradients = [&](int h, int qq) {
        const int q = iq[h], slot = islot[h];
        // the axis factors at point q: f[n][b] for a node with bit n = b
        double f[DIM][2];
#pragma unroll
        for (int n = 0; n < DIM; n++) {
            const bool up = (q >> n) & 1;
            f[n][1] = up ? kQ1Gp : kQ1Gm;
            f[n][0] = up ? kQ1Gm : kQ1Gp;
        }
#pragma unroll
        for (int k = 0; k < NEN; k++) {
            const int cb = q1_corner(k);
            double r[DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++) {
                double t = 1.0;
#pragma unroll
                for (int n = 0; n < DIM; n++)
                    if (n != m) t *= f[n][(cb >> n) & 1];
                r[m] = ((cb >> m) & 1) ? t : -t;
            }
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                double g = r[0] * G[h][a];
#pragma unroll
                for (int m = 1; m < DIM; m++) g = fma(r[m], G[h][m * DIM + a], g);
                sg[((qq * NEN + k) * DIM + a) * kGroupElems + slot] = se[h] * g;
            }
        }
    };
#pragma unroll
    for (int h = 1; h < kItems; h++)
        if (iq[h] < NQ) gradients(h, iq[h]);
    for (int pass = 0; pass < NPASS; pass++) {
        const int nqp = pass < NPASS - 1 ? QP : QLAST;
        const int qq = iq[0] - pass * QP;
        if (qq >= 0 && qq < nqp) gradients(0, qq);
        if (tid == 0) ticket = 0;
        __syncthreads();
        const int pmode = (pass > 0 ? kPassInit : 0) | (pass == NPASS - 1 ? kPassFinal : 0);
        if (pass < NPASS - 1) {
            if (gflags >> kGrpWideShift)
                assemble_wide<DIM, NEN, kF64, false, kGeoPoint + QP>(P, shdr, &ticket, stage, sg, nullptr, sn2l, lane,
                                                                     pmode);
            else
                assemble_pairs<DIM, NEN, kF64, false, kGeoPoint + QP>(P, shdr, &ticket, stage, sg, nullptr, sn2l,
                                                                      lane, pmode);
        } else {
            if (gflags >> kGrpWideShift)
                assemble_wide<DIM, NEN, kF64, false, kGeoPoint + QLAST>(P, shdr, &ticket, stage, sg, nullptr, sn2l,
                                                                        lane, pmode);
            else
                assemble_pairs<DIM, NEN, kF64, false, kGeoPoint + QLAST>(P, shdr, &ticket, stage, sg, nullptr, sn2l,
                                                                         lane, pmode);
        }
        __syncthreads();
    }
    store_rows<DIM, kStoreWaves>(P, shdr, srows, stage, w, lane);
}

// ---- per-point assembly with the partial sums in registers: work item r
// of a group (pairs, or wide for groups of at most 16 nodes) belongs to one
// wave for all passes, so a block's sum stays in the lane's registers across
// the passes and no stage holds partial sums; after the last pass the lane
// applies L and writes its block to K.  The contributions, their order and
// the lane layout are those of assemble_pairs / assemble_wide; a split
// position's two halves, and a wide item's phases, are added at the end.

// Pairs item r (r <= deg): this pass's terms of the lane's contributions
// into acc; with fin (after the last pass), the halves are added and the
// lane's block goes to its row block in the stage.
template <int DIM, int NEN, int QP>
__device__ __forceinline__ void point_pairs(const AsmParams &P, const int *hdr, int r, const double *Gs,
                                            const uint16_t *sn2l, int lane, double *stage, bool fin,
                                            double (&acc)[DIM][DIM]) {
    constexpr int NG = kGroupNodes;
    const int nn = wave_uniform(hdr[0]);
    const int deg = wave_uniform(hdr[1]);
    const int posoff = wave_uniform(hdr[2]);
    const int rkoff = wave_uniform(hdr[8]);
    const int rl = DIM * deg;
    const bool hi = lane >= NG;
    const int node = lane & (NG - 1);
    const uint16_t *n2l = sn2l + node;
    const int pa = ldc(P.sig_pairs, 2 * posoff + 2 * r);
    if (pa < 0) return;
    const int pb = ldc(P.sig_pairs, 2 * posoff + 2 * r + 1);
    const bool split = pb == pa;
    const int c0 = ldc(P.sig_pos_ptr, posoff + pa);
    const int na = ldc(P.sig_pos_ptr, posoff + pa + 1) - c0;
    int lo0 = c0, nlo = na, hi0 = c0, nhi = 0;
    if (split) {
        nlo = (na + 1) / 2;
        hi0 = c0 + nlo;
        nhi = na - nlo;
    } else if (pb >= 0) {
        hi0 = ldc(P.sig_pos_ptr, posoff + pb);
        nhi = ldc(P.sig_pos_ptr, posoff + pb + 1) - hi0;
    }
    if (!fin) {
        const int mycnt = hi ? nhi : nlo;
        const int32_t *lo_p = P.sig_contrib + lo0;
        const int32_t *hi_p = P.sig_contrib + (nhi > 0 ? hi0 : lo0);
        for (int t0 = 0; t0 < nlo; t0 += 8) {
            const Codes8 cl = ld_codes8(lo_p + t0), ch = ld_codes8(hi_p + t0);
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (t0 + u >= nlo) break;
                const bool oku = t0 + u < mycnt;
                const int code = oku ? (hi && nhi > 0 ? ch[u] : cl[u]) : 0;
                const int k = code >> 16, i = (code >> 8) & 255, j = code & 255;
                contribute_point<DIM, NEN, QP>(Gs, n2l[k * NG], i, j, oku, acc);
            }
        }
        return;
    }
    if (split) {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) acc[a][c] += __shfl_xor(acc[a][c], NG);
    }
    const int pme = hi ? pb : pa;
    if (node < nn && pme >= 0 && !(split && hi)) {
        const int pcsr = rkoff >= 0 ? (int)P.grp_rank[rkoff + pme * NG + node] : pme;
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; a++) tr += acc[a][a];
        double *dst = stage + node * wave_uniform(hdr[3]) + DIM * pcsr;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) {
                double o = P.lam * acc[a][c] + P.mu * acc[c][a];
                if (a == c) o += P.mu * tr;
                dst[a * rl + c] = o;
            }
    }
}

// Wide item r (r < number of wide items): as point_pairs, the phases of a
// position added by the butterfly at the end
template <int DIM, int NEN, int QP>
__device__ __forceinline__ void point_wide(const AsmParams &P, const int *hdr, int r, const double *Gs,
                                           const uint16_t *sn2l, int lane, double *stage, bool fin,
                                           double (&acc)[DIM][DIM]) {
    constexpr int NG = kGroupNodes;
    const int nn = wave_uniform(hdr[0]);
    const int deg = wave_uniform(hdr[1]);
    const int flags = wave_uniform(hdr[4]);
    const int wi0 = wave_uniform(hdr[5]);
    const int rkoff = wave_uniform(hdr[8]);
    const int lgN = 5 - ((flags >> kGrpWideShift) & 3);  // N = 8 or 16
    const int N = 1 << lgN;
    const int rl = DIM * deg;
    const int node = lane & (N - 1);
    const uint16_t *n2l = sn2l + node;
    const int32_t *rec = P.sig_witems + (int64_t)(wi0 + r) * kWideInts;
    const int np = ldc(rec, 0), Q = ldc(rec, 1), nt = ldc(rec, 2);
    const int lgQ = 31 - __clz(Q);
    const int grp = lane >> lgN;
    const int pp = grp >> lgQ, q = grp & (Q - 1);
    int p = -1, off = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (pp == k) {
            p = ldc(rec, 8 + k);
            off = ldc(rec, 16 + k);
            cnt = ldc(rec, 24 + k);
        }
    const bool mine = pp < np && node < nn;
    if (!fin) {
        int pk[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int ti = q + t * Q;
            pk[t] = (t < nt && mine && ti < cnt) ? P.sig_contrib[off + ti] : -1;
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
            if (t >= nt) break;
            if (pk[t] >= 0) {
                const int k = pk[t] >> 16, i = (pk[t] >> 8) & 255, j = pk[t] & 255;
                contribute_point<DIM, NEN, QP>(Gs, n2l[k * NG], i, j, true, acc);
            }
        }
        return;
    }
    for (int sh = N; sh < N * Q; sh <<= 1)
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) acc[a][c] += __shfl_xor(acc[a][c], sh);
    if (mine && q == 0) {
        const int pcsr = rkoff >= 0 ? (int)P.grp_rank[rkoff + p * NG + node] : p;
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; a++) tr += acc[a][a];
        double *dst = stage + node * wave_uniform(hdr[3]) + DIM * pcsr;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) {
                double o = P.lam * acc[a][c] + P.mu * acc[c][a];
                if (a == c) o += P.mu * tr;
                dst[a * rl + c] = o;
            }
    }
}

// Per-point assembly of Q1 elements (see k_assemble_quad) with the blocks'
// partial sums in registers: wave w owns work items w and w + NW (NW waves)
// for all passes, which holds for every plan whose signatures have at most
// 2 NW work items (the host checks; k_assemble_quad takes the others).  LDS
// holds the gradients of QP points, and after the last pass the finished
// blocks in a stage over the same bytes, so two workgroups share a CU and
// one's memory latency overlaps the other's arithmetic.  A block's
// sum: the passes in order; in a pass, the lane's contributions in the
// plan's order, each over the pass's points in order; then a split
// position's halves, or a wide item's phases, as in k_assemble.
template <int DIM>
struct PointShape {
    static constexpr int threads = DIM == 2 ? 256 : 512;
    static constexpr int qp = DIM == 2 ? 4 : 2;  // Gauss points per pass
    static constexpr int items = 2 * (threads / 64);  // work items a group may have
};

template <int DIM, int NEN>
__global__ __launch_bounds__(PointShape<DIM>::threads) void k_assemble_point(AsmParams P) {
    constexpr int kThreads = PointShape<DIM>::threads;
    constexpr int QP = PointShape<DIM>::qp;
    constexpr int NW = kThreads / 64;
    constexpr int D2 = DIM * DIM;
    constexpr int NQ = 1 << DIM;
    constexpr int NPASS = (NQ + QP - 1) / QP;
    static_assert(NQ % QP == 0, "equal passes");
    constexpr int NG = kGroupNodes;
    static_assert(NEN == NQ, "Q1 elements");
    static_assert(kGroupElems <= kThreads, "one thread per slot");
    extern __shared__ __align__(16) unsigned char smem[];
    // the gradients and, after the last pass, the stage in the same bytes
    double *sg = reinterpret_cast<double *>(smem);                  // [QP][NEN][DIM][kGroupElems]
    double *sE = sg + QP * NEN * DIM * kGroupElems;                 // [kGroupElems] sqrt(E(rho))
    int32_t *sid = reinterpret_cast<int32_t *>(sE + kGroupElems);  // [kGroupElems] column of qgeo
    double *stage = sg;                                             // [P.stage]
    const int64_t ubytes = (int64_t)(QP * NEN * DIM + 2) * kGroupElems * 8 > P.stage * 8
                               ? (int64_t)(QP * NEN * DIM + 2) * kGroupElems * 8
                               : P.stage * 8;
    int32_t *srows = reinterpret_cast<int32_t *>(smem + ubytes);    // [NG][2]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(srows + NG * 2);  // [kmax][NG]
    __shared__ int shdr[9];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int64_t NC = P.n_cells;
    const int ngr = P.n_groups;
    const int W = P.os_window;
    const int bid = blockIdx.x;
    const int base = bid - bid % W;
    const int gg = base + W <= ngr ? base + (bid % 8) * (W / 8) + (bid - base) / 8 : bid;
    if (gg >= ngr) return;
    const int sgi = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 0));
    const int eoff = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 2));
    const int ne = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 3));
    const int n2off = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 4));
    const int gflags = wave_uniform(ldc(P.grp_info, kGrpInfo * gg + 5));
    const int nk = wave_uniform(ldc(P.sig_info, 4 * sgi + 0)) * NG;
    for (int x = tid; x < nk; x += kThreads) sn2l[x] = P.grp_n2l[n2off + x];
    if (tid < 2 * NG) srows[tid] = P.grp_rows[(int64_t)gg * 2 * NG + tid];
    if (tid == 0) {
        shdr[0] = ldc(P.grp_info, kGrpInfo * gg + 1);
        shdr[1] = ldc(P.sig_info, 4 * sgi + 1);
        shdr[2] = ldc(P.sig_info, 4 * sgi + 2);
        shdr[3] = ldc(P.sig_info, 4 * sgi + 3);
        shdr[4] = gflags;
        const int wi0 = ldc(P.sig_witem_ptr, sgi);
        shdr[5] = wi0;
        shdr[6] = ldc(P.sig_witem_ptr, sgi + 1) - wi0;
        shdr[7] = -1;
        shdr[8] = P.grp_rank_off ? P.grp_rank_off[gg] : -1;
    }
    const bool wide = (gflags >> kGrpWideShift) != 0;
    double acc[2][DIM][DIM];
#pragma unroll
    for (int it = 0; it < 2; it++)
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) acc[it][a][c] = 0.0;
    // item (point qq of the pass, slot): the slot's gradients at that point,
    // sg[qq][k][a][slot] = g_k[a] = sqrt(E) sum_m grad phi_k(xi_q)[m]
    // G'_q[m][a]
    auto gradients = [&](const double (&G)[D2], double se, int q, int qq, int slot) {
        double f[DIM][2];
#pragma unroll
        for (int n = 0; n < DIM; n++) {
            const bool up = (q >> n) & 1;
            f[n][1] = up ? kQ1Gp : kQ1Gm;
            f[n][0] = up ? kQ1Gm : kQ1Gp;
        }
#pragma unroll
        for (int k = 0; k < NEN; k++) {
            const int cb = q1_corner(k);
            double r[DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++) {
                double t = 1.0;
#pragma unroll
                for (int n = 0; n < DIM; n++)
                    if (n != m) t *= f[n][(cb >> n) & 1];
                r[m] = ((cb >> m) & 1) ? t : -t;
            }
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                double g = r[0] * G[a];
#pragma unroll
                for (int m = 1; m < DIM; m++) g = fma(r[m], G[m * DIM + a], g);
                sg[((qq * NEN + k) * DIM + a) * kGroupElems + slot] = se * g;
            }
        }
    };
    auto modulus_root = [&](int id) {
        const int eo = P.elem_by_rank ? P.elem_by_rank[id] : id;
        return sqrt(P.Emin + simp_pow(static_cast<const double *>(P.rho)[eo], P.p, P.ip) * (P.E0 - P.Emin));
    };
    // one item per thread and pass (3D): the same slot in every pass, its
    // column and sqrt(E) kept in registers, and the next pass's G'_q read
    // while this pass's contributions are added
    constexpr bool kOneItem = QP * kGroupElems <= kThreads;
    const bool has = kOneItem && ne > 0 && tid < QP * ne;
    const int iqq = has ? tid / ne : 0, islot = has ? tid - iqq * ne : 0;
    int iid = 0;
    double ise = 0.0, Gc[D2], Gn[D2];
    if (has) {
        iid = P.grp_elems[eoff + islot];
        ise = modulus_root(iid);
#pragma unroll
        for (int c = 0; c < D2; c++) Gc[c] = P.qgeo[(int64_t)(iqq * D2 + c) * NC + iid];
    }
    for (int pass = 0; pass < NPASS; pass++) {
        if constexpr (kOneItem) {
            if (has) {
                gradients(Gc, ise, pass * QP + iqq, iqq, islot);
                if (pass + 1 < NPASS)
#pragma unroll
                    for (int c = 0; c < D2; c++) Gn[c] = P.qgeo[(int64_t)(((pass + 1) * QP + iqq) * D2 + c) * NC + iid];
            }
        } else {
            // several items per thread (2D: one pass)
            for (int x = tid; x < QP * ne; x += kThreads) {
                const int qq = x / ne, slot = x - qq * ne;
                const int q = pass * QP + qq;
                int id;
                double se;
                if (pass == 0) {
                    id = P.grp_elems[eoff + slot];
                    se = modulus_root(id);
                    if (qq == 0) {
                        sid[slot] = id;
                        sE[slot] = se;
                    }
                } else {
                    id = sid[slot];
                    se = sE[slot];
                }
                double G[D2];
#pragma unroll
                for (int c = 0; c < D2; c++) G[c] = P.qgeo[(int64_t)(q * D2 + c) * NC + id];
                gradients(G, se, q, qq, slot);
            }
        }
        __syncthreads();
        const int nitems = wide ? wave_uniform(shdr[6]) : wave_uniform(shdr[1]) + 1;
#pragma unroll
        for (int it = 0; it < 2; it++) {
            const int r = w + it * NW;
            if (r >= nitems) break;
            if (wide) point_wide<DIM, NEN, QP>(P, shdr, r, sg, sn2l, lane, stage, false, acc[it]);
            else point_pairs<DIM, NEN, QP>(P, shdr, r, sg, sn2l, lane, stage, false, acc[it]);
        }
        __syncthreads();
        if constexpr (kOneItem) {
#pragma unroll
            for (int c = 0; c < D2; c++) Gc[c] = Gn[c];
        }
    }
    // the blocks into the stage (over the gradients, read by now), then the
    // group's rows out as in k_assemble
    const int nitems = wide ? wave_uniform(shdr[6]) : wave_uniform(shdr[1]) + 1;
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const int r = w + it * NW;
        if (r >= nitems) break;
        if (wide) point_wide<DIM, NEN, QP>(P, shdr, r, sg, sn2l, lane, stage, true, acc[it]);
        else point_pairs<DIM, NEN, QP>(P, shdr, r, sg, sn2l, lane, stage, true, acc[it]);
    }
    __syncthreads();
    store_rows<DIM, NW>(P, shdr, srows, stage, w, lane);
}

// Dirichlet rows and columns (zero prescribed values): for a fixed dof r =
// DIM I + a, K[r, :] = 0, K[:, r] = 0, K[r, r] = 1.
//
// The writes of one fixed dof r by wave w of four, which takes the
// neighbours J = nb(I)[q], q = w, w + 4, ...  For each neighbour it writes
// the DIM entries of row r in J's columns and the DIM entries of column r in
// J's rows, the latter through the plan's transposed-slot table (slot of (row
// DIM J, column DIM I), degree of J).  J is I itself exactly when that slot
// is I's own block start + DIM q.  Where a row and a column write meet they
// write the same value, so the order of the writes does not matter.
template <int DIM>
__device__ __forceinline__ void dirichlet_dof(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ nb_tslot,
                                              const uint16_t *__restrict__ nb_tdeg, double *K, int r, int w) {
    const int I = r / DIM, a = r - DIM * I;
    const int b0 = row_ptr[r], b1 = row_ptr[r + 1];
    const int ib = row_ptr[DIM * I];  // first slot of node I's rows
    const int deg = (b1 - b0) / DIM;
    const int nptr = ib / (DIM * DIM);
    constexpr int B = 8;  // neighbours per thread with their loads in flight together
    for (int q0 = w; q0 < deg; q0 += 4 * B) {
        int ts[B], jl[B];
#pragma unroll
        for (int c = 0; c < B; c++) {
            const int q = q0 + 4 * c;
            ts[c] = q < deg ? nb_tslot[nptr + q] : 0;
            jl[c] = q < deg ? DIM * (int)nb_tdeg[nptr + q] : 0;
        }
#pragma unroll
        for (int c = 0; c < B; c++) {
            const int q = q0 + 4 * c;
            if (q < deg) {
                const bool self = ts[c] == ib + DIM * q;
#pragma unroll
                for (int e = 0; e < DIM; e++) {
                    const double v = (self && e == a) ? 1.0 : 0.0;
                    K[b0 + DIM * q + e] = v;           // row r, column DIM J + e
                    K[ts[c] + e * jl[c] + a] = v;      // row DIM J + e, column r
                }
            }
        }
    }
}

// The dofs are cut into chunks of 64 (lane = dof); workgroup b takes chunks
// b + k gridDim.x, k < kDirChunks (the launch makes kDirChunks gridDim.x
// cover every chunk), and loads all their mask bytes at once.  A mask with
// few fixed dofs thus costs few workgroups, and a contiguous run of fixed
// dofs (a clamped face) still spreads over many of them.
constexpr int kDirChunks = 8;
template <int DIM>
__global__ __launch_bounds__(256) void k_dirichlet(const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ nb_tslot,
                                                   const uint16_t *__restrict__ nb_tdeg,
                                                   const uint8_t *__restrict__ mask, double *K, int64_t ndof) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    uint8_t mk[kDirChunks];
#pragma unroll
    for (int k = 0; k < kDirChunks; k++) {
        const int64_t r64 = ((int64_t)blockIdx.x + (int64_t)k * gridDim.x) * 64 + lane;
        mk[k] = r64 < ndof ? mask[r64] : 0;
    }
    for (int k = 0; k < kDirChunks; k++) {
        if (!mk[k]) continue;
        const int r = (int)(((int64_t)blockIdx.x + (int64_t)k * gridDim.x) * 64 + lane);
        dirichlet_dof<DIM>(row_ptr, nb_tslot, nb_tdeg, K, r, w);
    }
}

// ------------------------------------------------------- element energies
//
// s_e = u_e^T K_e^0 u_e evaluated as the strain energy sum_q w_q |det J|
// (lambda tr(eps)^2 + 2 mu eps:eps) at the reference quadrature points (exact
// for affine elements; the same quadratic form as u_e^T K_e^0 u_e).
// Q1 elements, FP64: the reference gradient of u at the 2^d Gauss points of
// [0,1]^d by tensor-product factorisation.  The derivative along one axis does
// not depend on that axis' coordinate: it is the (bi)linear interpolation, in
// the other coordinates, of the nodal differences along the axis.  Energy
// lambda tr(eps)^2 + 2 mu eps:eps with eps = sym(grad_xi u G) at each point,
// equal weights.
template <class T>
__device__ __forceinline__ T q1_point_energy3(const T (&H)[3][3], const T (&G)[3][3], bool diag, T lam, T mu) {
    T eps[3][3];
    if (diag) {
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) eps[a][b] = H[a][b] * G[b][b];
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) eps[a][b] = H[a][0] * G[0][b] + H[a][1] * G[1][b] + H[a][2] * G[2][b];
    }
    const T tr = eps[0][0] + eps[1][1] + eps[2][2];
    const T h01 = T(0.5) * (eps[0][1] + eps[1][0]), h02 = T(0.5) * (eps[0][2] + eps[2][0]),
            h12 = T(0.5) * (eps[1][2] + eps[2][1]);
    const T ee = eps[0][0] * eps[0][0] + eps[1][1] * eps[1][1] + eps[2][2] * eps[2][2] +
                 T(2.0) * (h01 * h01 + h02 * h02 + h12 * h12);
    return lam * tr * tr + T(2.0) * mu * ee;
}

// AXIS: every element of the mesh is an axis-aligned box (diagonal J^-1),
// known from the plan; the per-element check and the full-G branch are then
// compiled out (the same arithmetic as the check's diagonal branch).  T is
// the arithmetic type: double, or float in the FP32 form (on displacements
// whose rigid motion was removed in FP64)
template <class T, bool AXIS>
__device__ __forceinline__ T q1_hex_energy(const T (&u)[8][3], const T (&G)[3][3], T lam, T mu) {
    // local node of corner (x, y, z): bottom face counter-clockwise, then top
    constexpr int N[2][2][2] = {{{0, 4}, {3, 7}}, {{1, 5}, {2, 6}}};
    const T gp[2] = {T(0.5 - 0.5 / 1.7320508075688772935), T(0.5 + 0.5 / 1.7320508075688772935)};
    const bool diag = AXIS || (G[0][1] == 0.0 && G[0][2] == 0.0 && G[1][0] == 0.0 && G[1][2] == 0.0 &&
                               G[2][0] == 0.0 && G[2][1] == 0.0);
    // d[ax][a][p][q]: nodal differences of u_a along axis ax, at the corners
    // (p, q) of the two other axes (in increasing axis order)
    T d[3][3][2][2];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int p = 0; p < 2; p++)
#pragma unroll
            for (int q = 0; q < 2; q++) {
                d[0][a][p][q] = u[N[1][p][q]][a] - u[N[0][p][q]][a];
                d[1][a][p][q] = u[N[p][1][q]][a] - u[N[p][0][q]][a];
                d[2][a][p][q] = u[N[p][q][1]][a] - u[N[p][q][0]][a];
            }
    auto lerp2 = [&](const T (&f)[2][2], T s, T t) {
        const T lo = f[0][0] + s * (f[1][0] - f[0][0]);
        const T hi = f[0][1] + s * (f[1][1] - f[0][1]);
        return lo + t * (hi - lo);
    };
    T sum = T(0.0);
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int k = 0; k < 2; k++) {
                T H[3][3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    H[a][0] = lerp2(d[0][a], gp[j], gp[k]);
                    H[a][1] = lerp2(d[1][a], gp[i], gp[k]);
                    H[a][2] = lerp2(d[2][a], gp[i], gp[j]);
                }
                sum += q1_point_energy3<T>(H, G, diag, lam, mu);
            }
    return T(0.125) * sum;
}

__device__ __forceinline__ double q1_quad_energy(const double (&u)[4][2], const double (&G)[2][2], double lam,
                                                 double mu) {
    constexpr int N[2][2] = {{0, 3}, {1, 2}};  // local node of corner (x, y)
    const double gp[2] = {0.5 - 0.5 / 1.7320508075688772935, 0.5 + 0.5 / 1.7320508075688772935};
    double D[2][2][2];  // D[axis][a][s]
#pragma unroll
    for (int a = 0; a < 2; a++) {
        const double dx0 = u[N[1][0]][a] - u[N[0][0]][a], dx1 = u[N[1][1]][a] - u[N[0][1]][a];
        const double dy0 = u[N[0][1]][a] - u[N[0][0]][a], dy1 = u[N[1][1]][a] - u[N[1][0]][a];
#pragma unroll
        for (int s = 0; s < 2; s++) {
            D[0][a][s] = dx0 + gp[s] * (dx1 - dx0);
            D[1][a][s] = dy0 + gp[s] * (dy1 - dy0);
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            double H[2][2], eps[2][2];
#pragma unroll
            for (int a = 0; a < 2; a++) {
                H[a][0] = D[0][a][j];
                H[a][1] = D[1][a][i];
            }
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++) eps[a][b] = H[a][0] * G[0][b] + H[a][1] * G[1][b];
            const double tr = eps[0][0] + eps[1][1];
            const double h = 0.5 * (eps[0][1] + eps[1][0]);
            const double ee = eps[0][0] * eps[0][0] + eps[1][1] * eps[1][1] + 2.0 * h * h;
            sum += lam * tr * tr + 2.0 * mu * ee;
        }
    return 0.25 * sum;
}

// Element energies on their own, one thread per element: dc_e =
// -E'(rho_e) s_e and a fixed-order block partial of sum_e E(rho_e) s_e.  In the
// FP32 form the element's rigid motion (translation of node 0 and the rotation
// of the centroid gradient) is removed in FP64 first; it is in the null space
// of K_e^0, so s_e is unchanged in exact arithmetic while the FP32 part sees
// only the deforming part.
template <int DIM, int NEN, int NQ, int PREC, bool AXIS>
__global__ __launch_bounds__(256) void k_energy(EnergyParams P) {
    __shared__ double red[256];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t NC = P.n_cells;
    constexpr int D2 = DIM * DIM;
    double cpart = 0.0;
    if (e < NC) {
        double G[DIM][DIM];
#pragma unroll
        for (int m = 0; m < DIM; m++)
#pragma unroll
            for (int a = 0; a < DIM; a++)
                G[m][a] = (AXIS && m != a) ? 0.0 : P.geo[(int64_t)(m * DIM + a) * NC + e];
        const double det = P.geo[(int64_t)D2 * NC + e];
        double u[NEN][DIM];
#pragma unroll
        for (int i = 0; i < NEN; i++) {
            const int n = P.cells[e * NEN + i];
#pragma unroll
            for (int a = 0; a < DIM; a++) u[i][a] = P.u[(int64_t)DIM * n + a];
        }
        double s = 0.0;
        if constexpr (PREC == kF64 && DIM == 3 && NEN == 8) {
            s = q1_hex_energy<double, AXIS>(u, G, P.lam, P.mu);
        } else if constexpr (PREC == kF64 && DIM == 2 && NEN == 4) {
            s = q1_quad_energy(u, G, P.lam, P.mu);
        } else if (PREC == kF64) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const double *dq = P.qgrad + q * NEN * DIM;
                double gr[DIM][DIM];  // reference gradient d u_a / d xi_m
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        double t = 0.0;
#pragma unroll
                        for (int i = 0; i < NEN; i++) t += u[i][a] * dq[i * DIM + m];
                        gr[a][m] = t;
                    }
                double eps[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        double t = 0.0;
#pragma unroll
                        for (int m = 0; m < DIM; m++) t += gr[a][m] * G[m][b];
                        eps[a][b] = t;
                    }
                double tr = 0.0, ee = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    tr += eps[a][a];
                    ee += eps[a][a] * eps[a][a];
#pragma unroll
                    for (int b = a + 1; b < DIM; b++) {
                        const double h = 0.5 * (eps[a][b] + eps[b][a]);
                        ee += 2.0 * h * h;
                    }
                }
                s += P.qw[q] * (P.lam * tr * tr + 2.0 * P.mu * ee);
            }
        } else {
            // FP64: remove translation (node 0) and the centroid rotation
            double w[NEN][DIM];
#pragma unroll
            for (int i = 0; i < NEN; i++)
#pragma unroll
                for (int a = 0; a < DIM; a++) w[i][a] = u[i][a] - u[0][a];
            const double *dc = P.cgrad;  // reference gradients at the centroid
            double gx[DIM][DIM];         // physical gradient at the centroid
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double t = 0.0;
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        double r = 0.0;
#pragma unroll
                        for (int i = 0; i < NEN; i++) r += w[i][a] * dc[i * DIM + m];
                        t += r * G[m][b];
                    }
                    gx[a][b] = t;
                }
            // x_i - x_0 = J xi_i, J = G^-1; W J xi_i with W = skew(gx)
            double J[DIM][DIM];
            if (DIM == 2) {
                const double d = G[0][0] * G[1][1] - G[0][1] * G[1][0];
                J[0][0] = G[1][1] / d; J[0][1] = -G[0][1] / d;
                J[1][0] = -G[1][0] / d; J[1][1] = G[0][0] / d;
            } else {
                // J = G^-1, i.e. (det J) * adj(G) with 1/det(G) = det J
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        const int a1 = (m + 1) % 3, a2 = (m + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
                        J[a][m] = det * (G[a1][b1] * G[a2][b2] - G[a1][b2] * G[a2][b1]);
                    }
            }
            double WJ[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int m = 0; m < DIM; m++) {
                    double t = 0.0;
#pragma unroll
                    for (int b = 0; b < DIM; b++) t += 0.5 * (gx[a][b] - gx[b][a]) * J[b][m];
                    WJ[a][m] = t;
                }
            float wf[NEN][DIM];
#pragma unroll
            for (int i = 0; i < NEN; i++)
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    double t = w[i][a];
#pragma unroll
                    for (int m = 0; m < DIM; m++) t -= WJ[a][m] * P.xref[i * DIM + m];
                    wf[i][a] = (float)t;
                }
            float Gf[DIM][DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int a = 0; a < DIM; a++) Gf[m][a] = (float)G[m][a];
            float sf = 0.0f;
            if constexpr (DIM == 3 && NEN == 8) {
                // Q1 hexahedra: the tensor-product form of the FP64 path, in
                // FP32 (the strains still formed at each Gauss point)
                sf = q1_hex_energy<float, AXIS>(wf, Gf, (float)P.lam, (float)P.mu);
            } else {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const float *dq = P.qgrad32 + q * NEN * DIM;
                float gr[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        float t = 0.0f;
#pragma unroll
                        for (int i = 0; i < NEN; i++) t += wf[i][a] * dq[i * DIM + m];
                        gr[a][m] = t;
                    }
                float eps[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        float t = 0.0f;
#pragma unroll
                        for (int m = 0; m < DIM; m++) t += gr[a][m] * Gf[m][b];
                        eps[a][b] = t;
                    }
                float tr = 0.0f, ee = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    tr += eps[a][a];
                    ee += eps[a][a] * eps[a][a];
#pragma unroll
                    for (int b = a + 1; b < DIM; b++) {
                        const float h = 0.5f * (eps[a][b] + eps[b][a]);
                        ee += 2.0f * h * h;
                    }
                }
                sf += (float)P.qw[q] * ((float)P.lam * tr * tr + 2.0f * (float)P.mu * ee);
            }
            }
            s = (double)sf;
        }
        s *= det;
        const double r = load_rho<PREC>(P.rho, e);
        const double rp1 = simp_pow(r, P.p - 1.0, P.ip >= 1 ? P.ip - 1 : -1);
        const double E = P.Emin + rp1 * r * (P.E0 - P.Emin);
        if (P.dc) store_out<PREC>(P.dc, e, -P.p * rp1 * (P.E0 - P.Emin) * s);
        cpart = E * s;
    }
    if (!P.partials) return;
    // compliance: fixed-order block partials of c and f^T u; wave_finalize
    // adds them in index order (k_finalize, or the assembly kernel of the
    // fused step).  (A last-block-done reduction in this kernel would need a
    // device-scope release per block, i.e. an L2 write-back on this chip,
    // which costs more than the extra launch.)
    double fpart = 0.0;
    if (P.f)
        for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < P.ndof; r += (int64_t)gridDim.x * 256)
            fpart += P.f[r] * P.u[r];
    const int nb = gridDim.x;
    // the block's two sums in block_sum_256's order with one barrier: the 256
    // values of each go to LDS, then wave 0 adds them as that tree does (lane
    // l holds threads l, l + 64, l + 128 and l + 192; the first two levels in
    // registers, the rest as shuffles)
    __shared__ double redf[256];
    red[threadIdx.x] = cpart;
    redf[threadIdx.x] = fpart;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        double xc = (red[l] + red[l + 128]) + (red[l + 64] + red[l + 192]);
        double xf = (redf[l] + redf[l + 128]) + (redf[l + 64] + redf[l + 192]);
        for (int st = 32; st > 0; st >>= 1) {
            xc += __shfl_down(xc, st);
            xf += __shfl_down(xf, st);
        }
        if (l == 0) {
            P.partials[blockIdx.x] = xc;
            P.partials[nb + blockIdx.x] = P.f ? xf : 0.0;
        }
    }
}

// c from the energy kernel's block partials: one wave (the fused step runs
// the same function inside the assembly kernel instead)
__global__ __launch_bounds__(64) void k_finalize(const double *__restrict__ partials, int n, int with_f, double *c) {
    wave_finalize(partials, n, with_f, c, threadIdx.x);
}

// ------------------------------------------------------------------ backward
//
// drho_e = E'(rho_e) sum_ij <Kbar(i,j), K_e^0(i,j)>
//        = E'(rho_e) |det J| sum_ij <L(X_ij), G^T M_ij G>
//        = E'(rho_e) |det J| sum_ij sum_mn M_ij[m][n] (G L(X_ij) G^T)[m][n],
// X_ij the stored Kbar block of (cells[e][i], cells[e][j]); L is self-adjoint.
template <int DIM, int NEN, int PREC>
__global__ __launch_bounds__(256) void k_backward(BwdParams P) {
    using T = typename CT<PREC>::T;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= P.n_cells) return;
    const int64_t NC = P.n_cells;
    constexpr int D2 = DIM * DIM;
    T G[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; m++)
#pragma unroll
        for (int a = 0; a < DIM; a++) G[m][a] = (T)P.geo[(int64_t)(m * DIM + a) * NC + e];
    const double det = P.geo[(int64_t)D2 * NC + e];
    int node[NEN], base[NEN], rowlen[NEN];
#pragma unroll
    for (int i = 0; i < NEN; i++) {
        node[i] = P.cells[e * NEN + i];
        base[i] = P.row_ptr[DIM * node[i]];
        rowlen[i] = P.row_ptr[DIM * node[i] + 1] - base[i];
    }
    const T lam = (T)P.lam, mu = (T)P.mu;
    double acc = 0.0;
    for (int i = 0; i < NEN; i++) {
        for (int j = 0; j < NEN; j++) {
            const int p = P.pos[(e * NEN + i) * NEN + j];
            T X[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double x = P.Kbar[base[i] + a * rowlen[i] + DIM * p + b];
                    if (P.mask && (P.mask[DIM * node[i] + a] | P.mask[DIM * node[j] + b])) x = 0.0;
                    X[a][b] = (T)x;
                }
            T tr = 0;
#pragma unroll
            for (int a = 0; a < DIM; a++) tr += X[a][a];
            T Y[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) Y[a][b] = lam * X[a][b] + mu * X[b][a] + (a == b ? mu * tr : T(0));
            T GY[DIM][DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    T t = 0;
#pragma unroll
                    for (int a = 0; a < DIM; a++) t += G[m][a] * Y[a][b];
                    GY[m][b] = t;
                }
            T blk = 0;
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int n = 0; n < DIM; n++) {
                    T z = 0;
#pragma unroll
                    for (int b = 0; b < DIM; b++) z += GY[m][b] * G[n][b];
                    const T Mv = PREC == kF64 ? (T)P.M[(i * NEN + j) * D2 + m * DIM + n]
                                              : (T)P.M32[(i * NEN + j) * D2 + m * DIM + n];
                    blk += Mv * z;
                }
            acc += (double)blk;
        }
    }
    const double r = load_rho<PREC>(P.rho, e);
    const double dE = P.p * simp_pow(r, P.p - 1.0, P.ip >= 1 ? P.ip - 1 : -1) * (P.E0 - P.Emin);
    store_out<PREC>(P.drho, e, dE * det * acc);
}

// ---------------------------------------------------------------- launchers

template <int DIM, int NEN, int PREC, bool FUSE>
static hipError_t launch_assemble_t(const AsmParams &P, int64_t ngroups, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = assemble_lds_bytes(DIM, NEN, PREC, P.stage, P.kmax);
    if (lds + 64 > 160 * 1024) return hipErrorInvalidValue;  // dynamic + static LDS
    const void *fn = reinterpret_cast<const void *>(&k_assemble<DIM, NEN, PREC, FUSE>);
    // the dynamic LDS limit only grows (per device, to the largest size
    // requested so far); the occupancy query runs once per device and size
    static std::mutex mu;
    static std::map<int, size_t> lds_limit;
    static std::map<std::pair<int, size_t>, int> occupancy;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        size_t &lim = lds_limit[dev];
        if (lds > lim) {
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            lim = lds;
        }
        auto it = occupancy.find({dev, lds});
        if (it != occupancy.end()) {
            per_cu = it->second;
        } else {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kAsmThreads, lds);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            occupancy[{dev, lds}] = per_cu;
        }
    }
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    const int64_t grid = std::min<int64_t>(ngroups, (int64_t)per_cu * ncu);
    hipLaunchKernelGGL((k_assemble<DIM, NEN, PREC, FUSE>), dim3((unsigned)grid), dim3(kAsmThreads), lds, st, P);
    return hipGetLastError();
}

static std::atomic<int> g_asm_variant{-1};
void set_assembly_variant(int v) { g_asm_variant.store(v); }

template <int DIM, int NEN, int PREC, bool FUSE>
static hipError_t launch_assemble_os_t(const AsmParams &P0, int64_t ngroups, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const size_t csz = PREC == kF64 ? 8 : 4;
    const size_t lds = 8 * (size_t)P0.stage + csz * DIM * DIM * kGroupElems + csz * NEN * NEN * DIM * DIM +
                       kGroupNodes * 2 * 4 + 2 * (size_t)P0.kmax * kGroupNodes;
    if (lds + 64 > 160 * 1024) return hipErrorInvalidValue;
    const void *fn = reinterpret_cast<const void *>(&k_assemble_os<DIM, NEN, PREC, FUSE>);
    static std::mutex mu;
    static std::map<int, size_t> lds_limit;
    static std::map<std::pair<int, size_t>, int> occupancy;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        size_t &lim = lds_limit[dev];
        if (lds > lim) {
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            lim = lds;
        }
        auto it = occupancy.find({dev, lds});
        if (it != occupancy.end()) {
            per_cu = it->second;
        } else {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, OsShape<DIM>::threads, lds);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            occupancy[{dev, lds}] = per_cu;
        }
    }
    AsmParams P = P0;
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    P.os_window = std::max(8, (per_cu * ncu) / 8 * 8);
    hipLaunchKernelGGL((k_assemble_os<DIM, NEN, PREC, FUSE>), dim3((unsigned)ngroups), dim3(OsShape<DIM>::threads),
                       lds, st, P);
    return hipGetLastError();
}

// The one-shot kernel where a group's stage is small (2D elements: many
// workgroups per CU overlap their loads, compute and stores) or where there
// are no more groups than two per CU (no steps for a persistent workgroup to
// pipeline); the persistent kernel otherwise.  Measured on MI355X: P1
// triangles 600x200 20 vs 33 us, Q1 quads 512^2 37 vs 60 us, Q1 hexahedra
// 16^3 11.1 vs 11.9 us; the 3D cantilever 115 vs 93 us, P2 box 730 vs 697 us.
template <int DIM, int NEN, int PREC, bool FUSE>
static hipError_t launch_assemble_v(const AsmParams &P, int64_t ngroups, hipStream_t st) {
    const int v = g_asm_variant.load();
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    const bool os = v == 1 || (v < 0 && (8 * P.stage <= 32768 || ngroups <= 2 * (int64_t)ncu));
    if (os) return launch_assemble_os_t<DIM, NEN, PREC, FUSE>(P, ngroups, st);
    return launch_assemble_t<DIM, NEN, PREC, FUSE>(P, ngroups, st);
}

hipError_t launch_assemble(int elem, int prec, const AsmParams &P, int64_t ngroups, hipStream_t st, bool fuse) {
#define SOPTX_ASM(E, D, N)                                                                     \
    case E:                                                                                    \
        if (fuse) {                                                                            \
            if (prec == kF64) return launch_assemble_v<D, N, kF64, true>(P, ngroups, st);      \
            return launch_assemble_v<D, N, kF32, true>(P, ngroups, st);                        \
        }                                                                                      \
        if (prec == kF64) return launch_assemble_v<D, N, kF64, false>(P, ngroups, st);         \
        return launch_assemble_v<D, N, kF32, false>(P, ngroups, st);
    switch (elem) {
        SOPTX_ASM(SOPTX_QUAD4, 2, 4)
        SOPTX_ASM(SOPTX_TRI3, 2, 3)
        SOPTX_ASM(SOPTX_HEX8, 3, 8)
        SOPTX_ASM(SOPTX_TET10, 3, 10)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_ASM
}

// LDS of k_assemble_quad for a plan's largest stage and slot table
static size_t quad_lds(int dim, int nen, int64_t stage, int kmax) {
    const int qp = dim == 2 ? QuadShape<2>::qp : QuadShape<3>::qp;
    return 8 * (size_t)stage + 8 * (size_t)qp * nen * dim * kGroupElems + kGroupNodes * 2 * 4 +
           2 * (size_t)kmax * kGroupNodes;
}

// LDS of k_assemble_point for a plan's slot table
static size_t point_lds(int dim, int nen, int64_t stage, int kmax) {
    const int qp = dim == 2 ? PointShape<2>::qp : PointShape<3>::qp;
    const size_t grad = 8 * (size_t)(qp * nen * dim + 2) * kGroupElems;  // with sqrt(E) and the columns
    return std::max(grad, 8 * (size_t)stage) + kGroupNodes * 2 * 4 + 2 * (size_t)kmax * kGroupNodes;
}

bool assemble_point_fits(int elem, int64_t stage, int kmax, int max_items) {
    if (elem != SOPTX_QUAD4 && elem != SOPTX_HEX8) return false;
    const int dim = elem == SOPTX_QUAD4 ? 2 : 3;
    const int items = dim == 2 ? PointShape<2>::items : PointShape<3>::items;
    return max_items <= items && point_lds(dim, 1 << dim, stage, kmax) + 64 <= 160 * 1024;
}

template <int DIM, int NEN>
static hipError_t launch_assemble_point_t(const AsmParams &P0, int64_t ngroups, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = point_lds(DIM, NEN, P0.stage, P0.kmax);
    if (lds + 64 > 160 * 1024) return hipErrorInvalidValue;
    const void *fn = reinterpret_cast<const void *>(&k_assemble_point<DIM, NEN>);
    static std::mutex mu;
    static std::map<int, size_t> lds_limit;
    static std::map<std::pair<int, size_t>, int> occupancy;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        size_t &lim = lds_limit[dev];
        if (lds > lim) {
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            lim = lds;
        }
        auto it = occupancy.find({dev, lds});
        if (it != occupancy.end()) {
            per_cu = it->second;
        } else {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PointShape<DIM>::threads, lds);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            occupancy[{dev, lds}] = per_cu;
        }
    }
    AsmParams P = P0;
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    P.os_window = std::max(8, (per_cu * ncu) / 8 * 8);
    hipLaunchKernelGGL((k_assemble_point<DIM, NEN>), dim3((unsigned)ngroups), dim3(PointShape<DIM>::threads), lds, st,
                       P);
    return hipGetLastError();
}

hipError_t launch_assemble_point(int elem, const AsmParams &P, int64_t ngroups, hipStream_t st) {
    if (!P.qgeo) return hipErrorInvalidValue;
    if (elem == SOPTX_QUAD4) return launch_assemble_point_t<2, 4>(P, ngroups, st);
    if (elem == SOPTX_HEX8) return launch_assemble_point_t<3, 8>(P, ngroups, st);
    return hipErrorInvalidValue;
}

bool assemble_quad_fits(int elem, int64_t stage, int kmax) {
    if (elem != SOPTX_QUAD4 && elem != SOPTX_HEX8) return false;
    const int dim = elem == SOPTX_QUAD4 ? 2 : 3;
    return quad_lds(dim, 1 << dim, stage, kmax) + 64 <= 160 * 1024;
}

template <int DIM, int NEN>
static hipError_t launch_assemble_quad_t(const AsmParams &P0, int64_t ngroups, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = quad_lds(DIM, NEN, P0.stage, P0.kmax);
    if (lds + 64 > 160 * 1024) return hipErrorInvalidValue;
    const void *fn = reinterpret_cast<const void *>(&k_assemble_quad<DIM, NEN>);
    static std::mutex mu;
    static std::map<int, size_t> lds_limit;
    static std::map<std::pair<int, size_t>, int> occupancy;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        size_t &lim = lds_limit[dev];
        if (lds > lim) {
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            lim = lds;
        }
        auto it = occupancy.find({dev, lds});
        if (it != occupancy.end()) {
            per_cu = it->second;
        } else {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, QuadShape<DIM>::threads, lds);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            occupancy[{dev, lds}] = per_cu;
        }
    }
    AsmParams P = P0;
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    P.os_window = std::max(8, (per_cu * ncu) / 8 * 8);
    hipLaunchKernelGGL((k_assemble_quad<DIM, NEN>), dim3((unsigned)ngroups), dim3(QuadShape<DIM>::threads), lds, st, P);
    return hipGetLastError();
}

hipError_t launch_assemble_quad(int elem, const AsmParams &P, int64_t ngroups, hipStream_t st) {
    if (!P.qgeo) return hipErrorInvalidValue;
    if (elem == SOPTX_QUAD4) return launch_assemble_quad_t<2, 4>(P, ngroups, st);
    if (elem == SOPTX_HEX8) return launch_assemble_quad_t<3, 8>(P, ngroups, st);
    return hipErrorInvalidValue;
}

template <int DIM, int NEN, int NQ, int PREC>
static hipError_t launch_energy_t(const EnergyParams &P, hipStream_t st) {
    unsigned nb = (unsigned)((P.n_cells + 255) / 256);
    if (nb == 0 && P.partials) nb = 1;  // c (and f^T u) still written
    if (nb == 0) return hipSuccess;
    // Q1 hexahedra, all axis-aligned: without the full-G branch the FP64
    // kernel needs 154 VGPRs instead of 188, three waves per SIMD instead of
    // two, and a 120x40x40 mesh's 750 blocks run in one round instead of two
    if constexpr (DIM == 3 && NEN == 8) {
        if (P.axis_aligned) {
            hipLaunchKernelGGL((k_energy<DIM, NEN, NQ, PREC, true>), dim3(nb), dim3(256), 0, st, P);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_energy<DIM, NEN, NQ, PREC, false>), dim3(nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_energy(int elem, int prec, const EnergyParams &P, hipStream_t st) {
    const int pr = prec == kF64 ? kF64 : kF32;
#define SOPTX_EN(E, D, N, Q)                                               \
    case E:                                                                \
        if (pr == kF64) return launch_energy_t<D, N, Q, kF64>(P, st);      \
        return launch_energy_t<D, N, Q, kF32>(P, st);
    switch (elem) {
        SOPTX_EN(SOPTX_QUAD4, 2, 4, 4)
        SOPTX_EN(SOPTX_TRI3, 2, 3, 1)
        SOPTX_EN(SOPTX_HEX8, 3, 8, 8)
        SOPTX_EN(SOPTX_TET10, 3, 10, 4)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_EN
}

hipError_t launch_dirichlet(int dim, const int32_t *row_ptr, const int32_t *nb_tslot, const uint16_t *nb_tdeg,
                            const uint8_t *mask, double *K, int64_t ndof, hipStream_t st) {
    const unsigned nb = (unsigned)(((ndof + 63) / 64 + kDirChunks - 1) / kDirChunks);
    if (nb == 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(k_dirichlet<2>, dim3(nb), dim3(256), 0, st, row_ptr, nb_tslot, nb_tdeg, mask, K, ndof);
    else hipLaunchKernelGGL(k_dirichlet<3>, dim3(nb), dim3(256), 0, st, row_ptr, nb_tslot, nb_tdeg, mask, K, ndof);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int n, int with_f, double *c, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, partials, n, with_f, c);
    return hipGetLastError();
}


template <int DIM, int NEN, int PREC>
static hipError_t launch_backward_t(const BwdParams &P, hipStream_t st) {
    const unsigned nb = (unsigned)((P.n_cells + 255) / 256);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_backward<DIM, NEN, PREC>), dim3(nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_backward(int elem, int prec, const BwdParams &P, hipStream_t st) {
    const int pr = prec == kF64 ? kF64 : kF32;
#define SOPTX_BW(E, D, N)                                          \
    case E:                                                        \
        if (pr == kF64) return launch_backward_t<D, N, kF64>(P, st); \
        return launch_backward_t<D, N, kF32>(P, st);
    switch (elem) {
        SOPTX_BW(SOPTX_QUAD4, 2, 4)
        SOPTX_BW(SOPTX_TRI3, 2, 3)
        SOPTX_BW(SOPTX_HEX8, 3, 8)
        SOPTX_BW(SOPTX_TET10, 3, 10)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_BW
}

// ------------------------------------------------ allocation-free evaluate
//
// Fixed device scratch of soptx_evaluate_noalloc: the block partials of c and
// of f^T u, 2 x kNoAllocBlocks doubles (128 KiB).  Every device that loads the
// library holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, not a device address: the device address comes
// from hipGetSymbolAddress, once per device with that device current, and
// only that address is passed to kernels.
static __device__ __align__(256) double scratch[2 * kNoAllocBlocks];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device -> address of its scratch
}  // namespace

hipError_t noalloc_scratch(int device, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double *>(p);
    *out = static_cast<double *>(p);
    return hipSuccess;
}

}  // namespace soptx
