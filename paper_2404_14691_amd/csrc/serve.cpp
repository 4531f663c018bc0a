// Serving loop (continuous batching with admission by free pool memory).
#include "internal.h"
