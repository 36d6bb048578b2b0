// Serving loop (continuous batching of render and inverse-optimisation requests).
#pragma once
#include "ctx.h"

void serve_shutdown(dist_ctx* ctx);
