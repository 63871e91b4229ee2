// Built-in launch shapes for gfx950 (MI355X): the table hif_tuning_get
// returns until hif_tuning_set replaces it.  Written by
// paper_1307_2666_amd/tune.py from timings on one MI355X; see that script for
// the candidates and the problem sizes of each bucket.
#pragma once

// waves per problem of the register-resident pivoted QR, problems of at most
// 64, 128 and 192 columns
#define HIF_TUNED_ID_REG_WAVES {4, 8, 16}
// threads of the register-resident LU panel, panels of at most 512 and 1024 rows
#define HIF_TUNED_LU_PANEL_THREADS {256, 512}
