/*
 * FP64 CPU oracle for the two sparse-Tucker products of LiFE.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; it exists so that tests, the smoke check and the CPU-baseline leg of
 * the benchmark can compare the HIP library against a plain, obviously correct
 * definition.  It shares no code, header or table with the HIP library.
 *
 * The matrix M (N_theta*N_v x N_f) of the LiFE model y ~ M w (Sec. 2.1, eq. 1) is
 * never formed.  With the sparse Tucker encoding M_v = S0(v) D Phi_v (eq. 3;
 * S0 is folded into the Phi values) and the tensor form Y = Phi x1 D x2 S0 x3 w^T
 * (eq. 4), a column block of M restricted to voxel v is D times the sparse
 * Na x Nf matrix Phi_v.  Phi is given as one (atom, voxel, fascicle, value) entry
 * per nonzero (Sec. 2.2).  The two products every SBB-NNLS iteration needs are:
 *
 *   DSC  y = M w :   y[t + Nt*v] = sum over nonzeros c with voxel_c = v of
 *                                  D[t + Nt*atom_c] * phi_c * w[fascicle_c]
 *   WC   g = M^T y:  g[f]        = sum over nonzeros c with fascicle_c = f of
 *                                  phi_c * sum_t D[t + Nt*atom_c] * y[t + Nt*voxel_c]
 *
 * Layouts: D and y are "vectors" indexed theta-fastest (offset Nt*index, Sec. 4.1,
 * removal of redundant offset computation).  Indices are 0-based.
 *
 * Both loops run over the nonzeros in the order given (no restructuring, no
 * partitioning), in double precision, exactly as the definitions read.
 */
#include <stdint.h>
#include <string.h>

/* y = M w  (eq. 1 with eq. 3/4).  y is overwritten. */
void oracle_dsc(int64_t nnz, int32_t n_theta, int32_t n_voxels,
                const int16_t *atom, const int32_t *voxel, const int32_t *fascicle,
                const double *phi, const double *D, const double *w, double *y)
{
    memset(y, 0, sizeof(double) * (size_t)n_theta * (size_t)n_voxels);
    for (int64_t c = 0; c < nnz; ++c) {
        const double s = phi[c] * w[fascicle[c]];
        const double *d = D + (int64_t)n_theta * atom[c];
        double *yv = y + (int64_t)n_theta * voxel[c];
        for (int32_t t = 0; t < n_theta; ++t)
            yv[t] += d[t] * s;
    }
}

/* g = M^T y  (the transpose product of eq. 6).  g is overwritten. */
void oracle_wc(int64_t nnz, int32_t n_theta, int32_t n_fascicles,
               const int16_t *atom, const int32_t *voxel, const int32_t *fascicle,
               const double *phi, const double *D, const double *y, double *g)
{
    memset(g, 0, sizeof(double) * (size_t)n_fascicles);
    for (int64_t c = 0; c < nnz; ++c) {
        const double *d = D + (int64_t)n_theta * atom[c];
        const double *yv = y + (int64_t)n_theta * voxel[c];
        double dot = 0.0;
        for (int32_t t = 0; t < n_theta; ++t)
            dot += d[t] * yv[t];
        g[fascicle[c]] += phi[c] * dot;
    }
}

/* Gradient of <ybar, M(D) w> with respect to the dictionary.  y = M(D) w is
 * linear in D (eq. 3/4: each nonzero adds D[:, atom_c] * phi_c * w[f_c] to
 * voxel_c's signal), so
 *   dD[t + Nt*a] = sum over nonzeros c with atom_c = a of
 *                  phi_c * w[fascicle_c] * ybar[t + Nt*voxel_c].
 * (The paper fits w only; this is the derivative a learned dictionary needs.)
 * dD (Nt*Na) is overwritten. */
void oracle_dd(int64_t nnz, int32_t n_theta, int32_t n_atoms,
               const int16_t *atom, const int32_t *voxel, const int32_t *fascicle,
               const double *phi, const double *w, const double *ybar, double *dD)
{
    memset(dD, 0, sizeof(double) * (size_t)n_theta * (size_t)n_atoms);
    for (int64_t c = 0; c < nnz; ++c) {
        const double s = phi[c] * w[fascicle[c]];
        const double *yv = ybar + (int64_t)n_theta * voxel[c];
        double *d = dD + (int64_t)n_theta * atom[c];
        for (int32_t t = 0; t < n_theta; ++t)
            d[t] += s * yv[t];
    }
}
