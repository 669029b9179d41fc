// Internal accessors of the PAH context shared by the PAH translation units.
#pragma once
#include "pah.h"

const pah_desc& pah_ctx_desc(const pah_ctx* c);
const double* pah_ctx_dnu(const pah_ctx* c);   // null before pah_build_tables
