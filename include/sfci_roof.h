/* sfci_roof.h -- device ceilings of the operations the sigma kernels are
 * built from (libsfci.so).  Not part of the method: the measured roofs
 * against which a sigma launch's throughput is reported.
 *
 * sigma = H v is scatter/gather work plus integer hashing: no dense
 * contraction, so the ceilings that matter are HBM streaming, random 8-byte
 * gathers, FP64 atomic adds into HBM and FP64 atomic adds into LDS (the
 * target-owned tile kernel accumulates every term with one LDS add).
 *
 * One call runs every probe on the current device, on the given stream, and
 * synchronises it.  It allocates and frees its own device buffers
 * (big_bytes + 1 GiB + a few MB); SFCI_E_NOMEM if they do not fit.  Times
 * are HIP events around each kernel, best of three runs.  Rates are per
 * second over the whole device.  Returns SFCI_E_ARG for a NULL out or a
 * big_bytes below 128 MiB. */
#ifndef SFCI_ROOF_H
#define SFCI_ROOF_H

#include <stdint.h>

#include "sfci.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double copy_GBps;          /* 1 GiB device-to-device copy: (bytes read + bytes written) / time */
    double gather_Gops[3];     /* random 8-byte loads per ns from arrays of 2 MiB, 128 MiB, big_bytes */
    double atomic_Gops[3];     /* random FP64 atomic adds (global_atomic_add_f64) per ns, same three sizes */
    double lds_atomic_Gops[2]; /* FP64 LDS atomic adds (ds_add_f64) per ns: [0] lane-consecutive slots,
                                  [1] random slots of a 64 KiB tile */
    double lds_read_Gops;      /* random 8-byte LDS reads per ns within a 64 KiB tile */
    uint64_t big_bytes;        /* the third array size */
} sfci_roof;

/* stream: a hipStream_t (NULL = default stream). */
sfci_status sfci_roof_probe(uint64_t big_bytes, void* stream, sfci_roof* out);

#ifdef __cplusplus
}
#endif
#endif /* SFCI_ROOF_H */
