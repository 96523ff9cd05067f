// Host-side construction of the operators of SFFT-based homogenization
// (preprocessing, run once per grid / reference medium / geometry).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace qtt {
namespace host {

using zc = std::complex<double>;

// A host tensor train (or operator) core list.  TT cores are (r0, d, r1)
// row-major; operator cores (r0, dout, din, r1); diagonal operator cores
// (r0, d, r1).
struct HCore {
  int r0 = 1, dout = 1, din = 0, r1 = 1;  // din = 0: TT core or diagonal operator core
  std::vector<zc> v;
};
using HTT = std::vector<HCore>;

// TT-SVD of a dense real tensor with dims[0..L-1] (row-major, first index
// slowest): successive truncated SVDs, per-bond threshold
// delta / sqrt(L-1) * ||T||, rank clipped to cap.
HTT tt_svd_real(const std::vector<double>& T, const std::vector<int>& dims,
                double delta, int cap);

// TT-rounding of a host train whose cores carry a combined physical index
// (dout * max(din,1)); same rule as tt_svd_real.
void tt_round(HTT& x, double delta, int cap);

// Reduced QFT Q_n as a TTO (cores (r0, 2, 2, r1), out index first), by
// contracting the circuit layer by layer with SVD truncation.
HTT qn_tto(int n, double delta);

// Green operator in bounded factors, SFFT momentum order.  With the unit
// direction n = xi/|xi| (n = 0 at xi = 0) the direct-scheme operator acts as
//   u_j = tau_jk n_k,  s = n . u,  q = u/(2 mu0) - (c/2) n s,
//   eps_ij = n_i q_j + n_j q_i,   c = (lam0 + mu0)/(mu0 (lam0 + 2 mu0)),
// averaged over the two Nyquist representatives sigma (Hermitian
// symmetrisation).  All four maps share the spatial cores of the joint
// train of n^sigma_a (control index (sigma, a), 6 values):
//   U: tau (6 Voigt) -> u (sigma, j);   Sd: u -> s (sigma);
//   P: s -> p = n s (sigma, j);         E: q (sigma, j) -> eps (6 Voigt).
// Every factor is bounded by 1 pointwise, so truncation errors are not
// amplified between the steps.
struct GreenFactors {
  HTT U, Sd, P, E;
  double inv_2mu0 = 0.0, half_c = 0.0;
};
GreenFactors green_factors(int n, double lam0, double mu0, double delta);
// The two scalars of the Green step that depend on the reference medium:
// 1/(2 mu0) and (lam0 + mu0) / (2 mu0 (lam0 + 2 mu0)) (the factors U, Sd,
// P, E do not depend on it).
void green_scalars(double lam0, double mu0, double* inv_2mu0, double* half_c);

// Joint train of the unit directions n^sigma_a in momentum order (core 0
// of dimension 6 = (sigma, a)).
HTT direction_train(int n, double delta);
// The four factors from an already computed direction train.
GreenFactors green_factors_from(const HTT& nt, double lam0, double mu0);
// Momentum frequencies of one axis (SFFT order) and their other Nyquist
// representative: f[k] in (-N/2, N/2], f2[k] = f[k] except -f[k] at N/2.
void momentum_freqs(int n, std::vector<double>& f, std::vector<double>& f2);

// Staggered-grid Green operator (App. A, Table 3: forward differences
// kp = exp(i q) - 1 on the normal strains, backward km = 1 - exp(-i q) on
// the shears, q = 2 pi m / N at DFT index m = -rev(k) mod N of momentum
// index k).  With B the strain symbol of this gradient the operator is
// B (B^H C0 B)^-1 B^H; for isotropic C0 the acoustic tensor is
// mu0 |kp|^2 I + (lam0 + mu0) conj(kp) kp^T (|km_a| = |kp_a| and
// conj(km) = -kp), so with the unit vectors n = kp / |kp|, m = km / |kp|
// the operator acts as
//   u_k = -m_k tau_kk - sum_{j != k} n_j tau_kj,   s = n . u,   p = m s,
//   q = u / mu0 + c' p / mu0,   c' = (lam0 + mu0) / (lam0 + 2 mu0),
//   eps_kk = n_k q_k,   gamma_ij = m_j q_i + m_i q_j.
// The factors share the train of (n_a, m_a) (control index (t, a), 6
// values): U: 6 -> 3, Sd: 3 -> 1, P: 1 -> 3, E: 3 -> 6; in GreenFactors
// inv_2mu0 holds the weight of u (1/mu0) and half_c minus that of p.
// One axis's symbols in momentum order (kp, km as (re, im) pairs).
void staggered_symbols(int n, std::vector<double>& kp, std::vector<double>& km);
GreenFactors green_factors_staggered_from(const HTT& nt, double lam0, double mu0);
// Plane-strain direct Green operator (2D, Voigt 11, 22, 12) from the train
// of the unit directions n^sigma_a, a in {x, y} (control 2 sigma + a, 4
// values): the same four maps as the 3D factors, U: 3 -> 4, Sd: 4 -> 2,
// P: 2 -> 4, E: 4 -> 3, with the same two scalars (the plane-strain
// acoustic tensor is mu0 |xi|^2 I + (lam0 + mu0) xi xi^T on the plane).
GreenFactors green_factors2d_from(const HTT& nt, double lam0, double mu0);
// The plane staggered-grid factors (the 3D derivation restricted to the
// plane) from the train of (n_a, m_a), a in {x, y} (control 2 t + a):
// U: 3 -> 2, Sd: 2 -> 1, P: 1 -> 2, E: 2 -> 3, the staggered scalars.
GreenFactors green_factors_staggered2d_from(const HTT& nt, double lam0, double mu0);
// The Green step's two medium scalars for a scheme (0 direct, 1 staggered):
// q = a u - c p.
void green_scalars_scheme(int scheme, double lam0, double mu0, double* a, double* c);

// Raised stiffness operator C(x) - C0 (or one-hot phase train chi) from a
// voxel phase array; returns the operator, and the one-hot train in chi.
HTT stiffness_tto(const uint8_t* phase, int n, int nphase, const double* lame,
                  const double* lame0, double delta, int cap, HTT* chi,
                  int* max_rank);

// The same operator from an already computed one-hot phase train (core 0
// of dimension nphase, then the 3n binary cores); chi receives the train.
HTT stiffness_from_chi(HTT t, int nphase, const double* lame, const double* lame0, int cap, HTT* chi,
                       int* max_rank, int voigt = 6);

// Isotropic Voigt stiffness (order 11, 22, 33, 23, 13, 12).
void iso_voigt(double lam, double mu, double C[36]);
// The same for a Voigt dimension: 6, or 3 for plane strain (11, 22, 12:
// [[lam + 2 mu, lam, 0], [lam, lam + 2 mu, 0], [0, 0, mu]]), row-major.
void iso_voigt_dim(int voigt, double lam, double mu, double* C);

}  // namespace host
}  // namespace qtt
