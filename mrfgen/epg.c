/* Extended-phase-graph (EPG) simulation of a FISP fingerprint train.
 *
 * Input generator only: it produces the dictionary atoms d_m = B(eta_m; theta) that the
 * reconstruction takes as a precomputed input (eq. (3), Sec. II-B), and the noise-free
 * ground-truth fingerprints of the synthetic phantoms (eq. (2)). It implements no step of
 * the reconstruction itself.
 *
 * Model (Weigel, J. Magn. Reson. Imaging 2015): states F+_k, F-_k, Z_k, k = 0..K-1.
 * An ideal 180-degree inversion, one TR of recovery, then for each frame l:
 *   RF rotation by flip angle a_l * b1 about x, record F+_0 * exp(-TE/T2) as the signal,
 *   relax over TR (E1, E2, recovery into Z_0), then one dephasing shift of the F states
 *   (FISP: an unbalanced gradient per TR). States beyond K are dropped.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

void mrfgen_epg_fisp(int n_atoms, int n_frames, int n_states,
                     const double *t1, const double *t2, const double *b1,
                     const double *fa_deg, const double *tr_ms, double te_ms,
                     float *out /* [n_atoms][n_frames][2] interleaved complex64 */)
{
#pragma omp parallel
    {
        double complex *fp = malloc(sizeof(double complex) * n_states);
        double complex *fm = malloc(sizeof(double complex) * n_states);
        double complex *z = malloc(sizeof(double complex) * n_states);
        double complex *nfp = malloc(sizeof(double complex) * n_states);
        double complex *nfm = malloc(sizeof(double complex) * n_states);
#pragma omp for schedule(dynamic, 16)
        for (int m = 0; m < n_atoms; ++m) {
            const double T1 = t1[m], T2 = t2[m], scale = b1 ? b1[m] : 1.0;
            memset(fp, 0, sizeof(double complex) * n_states);
            memset(fm, 0, sizeof(double complex) * n_states);
            memset(z, 0, sizeof(double complex) * n_states);
            /* inversion, then recovery over one TR */
            {
                const double e1 = exp(-tr_ms[0] / T1);
                z[0] = -1.0 * e1 + (1.0 - e1);
            }
            const double e2te = exp(-te_ms / T2);
            for (int l = 0; l < n_frames; ++l) {
                const double a = fa_deg[l] * (M_PI / 180.0) * scale;
                const double c2 = cos(0.5 * a) * cos(0.5 * a), s2 = sin(0.5 * a) * sin(0.5 * a);
                const double sa = sin(a), ca = cos(a);
                const double e1 = exp(-tr_ms[l] / T1), e2 = exp(-tr_ms[l] / T2);
                for (int k = 0; k < n_states; ++k) {
                    const double complex p = fp[k], q = fm[k], w = z[k];
                    nfp[k] = c2 * p + s2 * q - I * sa * w;
                    nfm[k] = s2 * p + c2 * q + I * sa * w;
                    z[k] = -0.5 * I * sa * p + 0.5 * I * sa * q + ca * w;
                }
                const double complex sig = nfp[0] * e2te;
                out[2 * ((size_t)m * n_frames + l) + 0] = (float)creal(sig);
                out[2 * ((size_t)m * n_frames + l) + 1] = (float)cimag(sig);
                for (int k = 0; k < n_states; ++k) {
                    nfp[k] *= e2;
                    nfm[k] *= e2;
                    z[k] *= e1;
                }
                z[0] += 1.0 - e1;
                /* dephasing: F+ moves up one order, F- moves down one order */
                for (int k = n_states - 1; k >= 1; --k) fp[k] = nfp[k - 1];
                for (int k = 0; k < n_states - 1; ++k) fm[k] = nfm[k + 1];
                fm[n_states - 1] = 0.0;
                fp[0] = conj(fm[0]);
            }
        }
        free(fp); free(fm); free(z); free(nfp); free(nfm);
    }
}
