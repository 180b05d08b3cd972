/*
 * moa_hypercube.h -- C ABI of the hyper-cube kernels of the MI355X MoA
 * library: the generalized transpose of an array viewed as a hyper-cube of
 * 2-element axes, and the gating of a density matrix by direct indexing
 * through that view (Ch. 6, "Density Matrix Operations for a Quantum
 * Computer").  Same conventions as moa_fft.h: device pointers owned by the
 * caller, asynchronous on a HIP stream (NULL = null stream), a status code
 * from every call, arguments validated on the host before any HIP call.
 * Neither call allocates memory.
 */
#ifndef MOA_HYPERCUBE_H
#define MOA_HYPERCUBE_H

#include "moa_fft.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * out = t transpose (<2 2 ... 2> reshape in), ravelled: the array of 2^rank
 * elements viewed as a hyper-cube of `rank` axes of extent 2 (row-major:
 * axis 0 is the most significant bit of an element's offset), transposed in
 * the sense of Ch. 2 -- i psi (t transpose A) = i[t] psi A -- so that
 *     out[gamma(i; s)] = in[gamma(i[t]; s)],  i[t]_k = i[t_k],  s = <2 ... 2>
 * (the generic normal form of Ch. 6, "Final Expression and Normal Form";
 * the same movement as the reshape-transposes of Ch. 4, "Reordering the
 * Data").  Every element moves once: a pure data movement, elem_bytes bytes
 * per element (4, 8 or 16: e.g. float, complex64, complex128).
 *
 * rank: 1..34, with 2^rank * elem_bytes at most 2^38 bytes.  t: host array
 * of `rank` entries, a permutation of 0..rank-1.  in and out: device
 * buffers of 2^rank elements, 16-byte aligned, not overlapping (no in-place
 * form).  Errors: MOA_ERR_NULL (t, in or out NULL), MOA_ERR_SIZE (rank or
 * total size out of range), MOA_ERR_ARG (t not a permutation, elem_bytes
 * not 4/8/16, misaligned or overlapping buffers), MOA_ERR_HIP (launch).
 */
moa_status_t moa_hypercube_transpose(int32_t rank, const int32_t* t, int32_t elem_bytes, const void* in,
                                     void* out, void* stream);

/*
 * Gate q qubits of an n-qubit density matrix in place: rho <- G rho G^H,
 * where G is the gate matrix U on the gated qubits and the identity on the
 * others (Ch. 6, "Quantum Evolution: the Density Matrix"):
 *     G[i][j] = U[g(i)][g(j)] when i and j agree on every bit that is not
 *     gated, else 0,
 * g(i) packing the gated bits of i with the highest gated bit as the most
 * significant bit of U's index.  Computed as in "The Algorithm": the
 * matrix is viewed through the transpose that moves the gated bits to the
 * low bits of both indices (the block-diagonal arrangement), and every
 * 2^q x 2^q block B of that view becomes U B U^H -- by direct indexing of
 * rho through the normal form, with no permuted copy and no 2^n x 2^n gate
 * matrix.  (The paper multiplies "on the right and left by a unitary matrix
 * and its inverse"; G rho G^H is that statement for the gate U^H.)
 *
 * n_qubits: 1..15 (rho is 2^n x 2^n, row-major, complex64 or complex128
 * interleaved).  q: 1..4, at most n_qubits.  gated_bits: host array of q
 * distinct bit positions in [0, n_qubits), bit 0 the least significant bit
 * of a row or column index; their order in the array does not matter.
 * gate: device array of U, 2^q x 2^q row-major, same dtype as rho (U need
 * not be unitary: the call computes G rho G^H for any U).  rho: device
 * buffer, 16-byte aligned.  Errors: MOA_ERR_NULL, MOA_ERR_SIZE (n_qubits or
 * q out of range), MOA_ERR_ARG (a gated bit out of range or repeated,
 * misaligned rho), MOA_ERR_DTYPE, MOA_ERR_HIP.
 */
moa_status_t moa_density_gate(int32_t n_qubits, int32_t q, const int32_t* gated_bits, const void* gate,
                              moa_fft_dtype_t dtype, void* rho, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MOA_HYPERCUBE_H */
