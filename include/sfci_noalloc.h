/* sfci_noalloc.h -- an entry point of libsfci.so that allocates nothing.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * sfci_topm_noalloc is sfci_topm (see sfci.h: the truncation of Sec. 2.1,
 * Eqs. 10-11, by ascending rank, optional Eq. 11 division, optional tie band)
 * with all of its working memory in a fixed device array of the library
 * (about 60 KB, held on every device the library runs on until the process
 * ends) instead of buffers it allocates.  It calls no hipMalloc or hipFree.
 * The caller still passes the input v and the output out (device arrays,
 * caller-owned, as in sfci.h).
 *
 * Limits and errors: v->nnz may be at most SFCI_TOPM_NOALLOC_MAX_NNZ, else
 * SFCI_E_ARG; SFCI_E_RANGE / SFCI_E_DUP for ranks >= N_det / not strictly
 * ascending; SFCI_E_CAPACITY (out->nnz = the size needed) when out is too
 * small.  Runs on the problem's stream and synchronises it.
 *
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (two host threads, or two
 * streams) race and must be serialised by the caller. */
#ifndef SFCI_NOALLOC_H
#define SFCI_NOALLOC_H

#include <stdint.h>

#include "sfci.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SFCI_TOPM_NOALLOC_MAX_NNZ (1ull << 24)

sfci_status sfci_topm_noalloc(sfci_problem* prob, const sfci_svec* v, uint64_t M, int32_t normalise,
                              int32_t tie_band, sfci_svec* out);

#ifdef __cplusplus
}
#endif
#endif /* SFCI_NOALLOC_H */
