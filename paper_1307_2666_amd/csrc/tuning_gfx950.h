// Built-in launch shapes for gfx950 (MI355X): the table hif_tuning_get
// returns until hif_tuning_set replaces it.  Written by
// paper_1307_2666_amd/tune.py from timings on one MI355X; see that script for
// the candidates and the problem sizes of each bucket.
//
// Medians (ms):
//   ID, 4096 problems of 33-64 columns: 4 waves 0.851, 8 waves 0.915, 16 waves 1.033
//   ID, 2048 problems of 97-128 columns: 4 waves 3.013, 8 waves 2.362, 16 waves 2.730
//   ID, 1024 problems of 161-192 columns: 8 waves 4.344, 16 waves 3.403
//   LU, 256 blocks of 257-512 rows: 256 threads 3.092, 512 threads 2.959, 1024 threads 3.158
//   LU, 64 blocks of 513-1024 rows: 512 threads 6.269, 1024 threads 6.340
//   8-RHS solve of a 384 x 384 factorization: 64 threads 5.562, 128 threads 5.234, 256 threads 5.116
//   row compression of a 384 x 384 factorization (eps 1e-6): 4 waves 54.97, 8 waves 59.47, 4 waves + LDS 56.60, 8 waves + LDS 54.56, 4 waves rows split 57.59, 8 waves rows split 57.01
#pragma once

// waves per problem of the register-resident pivoted QR, problems of at most
// 64, 128 and 192 columns
#define HIF_TUNED_ID_REG_WAVES {4, 8, 16}
// threads of the register-resident LU panel, panels of at most 512 and 1024 rows
#define HIF_TUNED_LU_PANEL_THREADS {512, 512}
// waves (16 columns each) per workgroup of the row compression's trailing
// update beside the next panel
#define HIF_TUNED_ROWQR_UPDATE_WAVES 8
// 0: Y in registers, 1: the chunk reflectors staged in LDS, 2: rows split over two waves
#define HIF_TUNED_ROWQR_UPDATE_KIND 1
// threads per record of the sweeps on sub-levels of at least 1024 records
#define HIF_TUNED_SWEEP_MANY_THREADS 256
